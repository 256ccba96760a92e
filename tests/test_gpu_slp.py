"""GPU parity of the SLP step's LP subproblem (Sec. 4.1, problem (Pstar); the
artificial problem (Pstar2) when it has no solution) against the oracle,
through the C ABI.

Every entry of the step but the critical one is a bound (l or u), the same
FP64 value on both sides: at most one entry may differ.  The critical entry is
l_k + R / a_k, where R, the budget left for it, is B minus a sum of
capacities taken in another order than the oracle's: by the bound of
recursive summation the two R differ by at most 2 n eps (sum of the
capacities), so the entries by that over a_k.  The multiplier is the
critical ratio -g_k / a_k, the same FP64 quotient on both sides when both pick
the same variable: compared exactly.  g^T s and a^T s are sums of n products:
within n eps of the sum of the products' magnitudes."""

import numpy as np
import pytest

from oracle import slp
from tests.helpers import need_gpu

pytestmark = pytest.mark.gpu


def _instance(n, seed, delta=0.1, frac=0.37, ties=False):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    x[rng.random(n) < 0.1] = 0.0   # some variables at the bounds
    x[rng.random(n) < 0.1] = 1.0
    g = -rng.exponential(1.0, n) + 0.3 * rng.standard_normal(n)
    a = rng.uniform(0.5, 1.5, n)
    if ties:
        g = np.round(g, 1)
        a = np.ones(n)
    l, u = slp.lp_bounds(x, delta)
    b = float(a @ l + frac * (a @ (u - l)))
    return g, a, x, b, delta


def _check(g, a, x, b, delta, lp):
    s, info = lp.solve(g, a, x, b, delta)
    s_o, lam_o, ok_o = slp.lp_step(g, a, x, b, delta)
    n, eps = g.size, np.finfo(np.float64).eps
    assert info["feasible"] == ok_o
    l, u = slp.lp_bounds(x, delta if ok_o else 0.8 * delta)
    # at most the critical entry differs (its budget, even when the oracle's
    # is exactly 0 or the full capacity, carries the other summation order)
    diff = np.flatnonzero(s != s_o)
    assert diff.size <= 1, diff[:10]
    if diff.size:
        k = diff[0]
        capsum = float(np.sum(a * (u - l)))
        assert abs(s[k] - s_o[k]) <= 2 * n * eps * capsum / a[k]
    if ok_o:
        assert info["lambda"] == lam_o
        assert abs(info["ats"] - b) <= 2 * n * eps * float(np.abs(a * s_o).sum())
    assert abs(info["gts"] - float(g @ s_o)) <= 2 * n * eps * float(np.abs(g * s_o).sum())
    assert info["s_inf"] == pytest.approx(float(np.abs(s_o).max()), rel=1e-14)
    return s, info


@pytest.mark.parametrize("n,seed,frac,ties", [
    (1, 0, 0.5, False), (7, 1, 0.0, False), (255, 2, 0.37, False), (256, 3, 1.0, False),
    (257, 4, 0.9, False), (1000, 5, 0.37, True), (70001, 6, 0.61, False),
    (70001, 7, 0.2, True)])
def test_lp_matches_oracle(n, seed, frac, ties):
    need_gpu()
    from paper_2311_05595_amd import api
    lp = api.LP(n)
    g, a, x, b, delta = _instance(n, seed, frac=frac, ties=ties)
    _check(g, a, x, b, delta, lp)
    lp.close()


def test_lp_infeasible_and_bad_input():
    need_gpu()
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError
    n = 3000
    lp = api.LP(n)
    g, a, x, b, delta = _instance(n, 8)
    l, u = slp.lp_bounds(x, delta)
    for bb in (float(a @ l) - 1.0, float(a @ u) + 1.0):
        s, info = _check(g, a, x, bb, delta, lp)
        assert not info["feasible"] and np.isnan(info["lambda"])
    a_bad = a.copy()
    a_bad[17] = 0.0
    with pytest.raises(MGCGError):
        lp.solve(g, a_bad, x, b, delta)
    # the object stays usable
    _check(g, a, x, b, delta, lp)
    lp.close()


def test_lp_full_size_device_memory():
    """The design lattice of the 64x32x32 mesh with 2^3 design cells per
    element (524,288 variables), device vectors, the same bits as the
    host-memory path, and the oracle's solution."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    n = 64 * 32 * 32 * 8
    lp = api.LP(n)
    g, a, x, b, delta = _instance(n, 9, delta=0.05)
    s_h, info_h = _check(g, a, x, b, delta, lp)
    gd, ad, xd = (torch.tensor(v, device="cuda") for v in (g, a, x))
    s_d, info_d = lp.solve(gd, ad, xd, b, delta)
    assert np.array_equal(s_d.cpu().numpy(), s_h)
    assert info_d == info_h
    lp.close()


def test_slp_iterations_match_oracle():
    """Three iterations of Algorithm 2 on a small multiresolution cantilever
    (6x4x4 elements, 2^3 densities and one design variable per element,
    rmin = 1.1, V_max = 0.3 of the volume): projection, solve, compliance and
    gradient, the chain rule W^T, the LP step, the trial solve and the
    accept/reject decision, all through the library, against the same
    iterations composed from the oracle.  The designs agree to the solves'
    accuracy (rtol 1e-11)."""
    need_gpu()
    import torch
    import workloads as W
    from oracle import fem, projection as P, solve
    from paper_2311_05595_amd import api
    nel, n, d, rmin = (6, 4, 4), 2, 1, 1.1
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    prob = api.Problem(nel, mask, f, nsub=n, nlevels=2)
    pr = api.Projection(nel, n, d, rmin)
    lp = api.LP(pr.nx)
    rng = np.random.default_rng(5)
    x0 = rng.uniform(0.2, 0.4, pr.nx)
    vmax = 0.3 * np.prod(nel)
    v = np.full(pr.nrho, 1.0 / n ** 3)
    a = pr.apply_transpose(v)                      # volume gradient W^T v
    Wm = P.projection_matrix(nel, n, d, rmin)
    a_o = Wm.T @ v
    Ks = fem.sub_element_matrices(1, n)
    mat = dict(E0=1.0, Emin=1e-9, penal=3.0)

    def gpu_eval(x):
        prob.set_densities(pr.apply(x))
        prob.solve(rtol=1e-11, maxit=2000, warm_start=False)
        c, dc = prob.compliance_sensitivity()
        return c[-1], pr.apply_transpose(dc)

    def oracle_eval(x):
        rho = (Wm @ x).reshape(P.lattice_shape(nel, n))
        _, _, c, dc = solve.solve_problem(rho, mask, f, nel, 1, n, Ks, **mat)
        return c.sum(), Wm.T @ dc

    assert np.abs(a - a_o).max() <= 1e-13 * np.abs(a_o).max()
    xg, xo = x0.copy(), x0.copy()
    ctrl = api.slp_ctrl(0.1, delta_min=1e-3, box_inf=1.0)
    delta, tmax, hist, k = 0.1, 1.0, [1.0], 0
    fg, gg = gpu_eval(xg)
    fo, go = oracle_eval(xo)
    for it in range(3):
        assert abs(fg - fo) <= 1e-9 * fo
        # LP step at the current design
        cg = float(a @ xg) - vmax
        sg, info = lp.solve(gg, a, xg, -cg, ctrl.delta)
        co = float(a_o @ xo) - vmax
        so, lam_o, ok_o = slp.lp_step(go, a_o, xo, -co, delta)
        assert info["feasible"] == ok_o
        assert np.abs(sg - so).max() <= 1e-7 * delta
        # trial point and decision
        fg1, gg1 = gpu_eval(xg + sg)
        fo1, go1 = oracle_eval(xo + so)
        acc, th, ar, pr_ = api.slp_decide(ctrl, fg, fg1, cg, float(a @ (xg + sg)) - vmax,
                                          info["gts"], info["ats"], info["s_inf"])
        _, _, pf, po = slp.merit_reductions(1.0, fo, fo1, go, so, co,
                                            float(a_o @ (xo + so)) - vmax, a_o)
        th_o = slp.theta_update(k, hist, tmax, pf, po)
        ar_o, pr_o, _, _ = slp.merit_reductions(th_o, fo, fo1, go, so, co,
                                                float(a_o @ (xo + so)) - vmax, a_o)
        acc_o, delta = slp.trust_update(ar_o, pr_o, delta, float(np.abs(so).max()), 1.0, 1e-3)
        assert acc == acc_o and th == pytest.approx(th_o, rel=1e-6)
        assert ctrl.delta == pytest.approx(delta, rel=1e-6)
        if acc_o:
            xg, fg, gg = xg + sg, fg1, gg1
            xo, fo, go = xo + so, fo1, go1
            hist.append(th_o)
            tmax, k = 1.0, k + 1
        else:
            tmax = th_o
        assert np.abs(xg - xo).max() <= 1e-7
    assert k >= 1  # at least one step was taken
    lp.close()
    pr.close()
    prob.close()


@pytest.mark.parametrize("n,seed,frac,mem", [(257, 11, 0.37, "host"), (70001, 12, 0.55, "host"),
                                            (70001, 13, 0.2, "device"), (3000, 14, -1.0, "host")])
def test_lp_fixed_variables_match_oracle(n, seed, frac, mem):
    """Fixed design variables (Sec. 6.1) held at s = 0, against the oracle's
    LP with l = u = 0 there (frac < 0: an infeasible budget, the artificial
    problem)."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    g, a, x, b, delta = _instance(n, seed, frac=max(frac, 0.0))
    fixed = (np.random.default_rng(seed).random(n) < 0.3).astype(np.uint8)
    l, u = slp.lp_bounds(x, delta, fixed=fixed)
    b = float(a @ l + frac * (a @ (u - l))) if frac >= 0 else float(a @ l) - 1.0
    lp = api.LP(n)
    if mem == "device":
        t = lambda v: torch.tensor(v, device="cuda")
        s, info = lp.solve(t(g), t(a), t(x), b, delta, fixed=t(fixed))
        s = s.cpu().numpy()
    else:
        s, info = lp.solve(g, a, x, b, delta, fixed=fixed)
    s_o, lam_o, ok_o = slp.lp_step(g, a, x, b, delta, fixed=fixed)
    assert info["feasible"] == ok_o
    assert np.all(s[fixed == 1] == 0.0)
    diff = np.flatnonzero(s != s_o)
    assert diff.size <= 1
    if diff.size:
        k = diff[0]
        l2, u2 = slp.lp_bounds(x, delta, fixed=fixed)
        assert abs(s[k] - s_o[k]) <= 2 * n * np.finfo(float).eps * float(np.sum(a * (u2 - l2))) / a[k]
    if ok_o:
        assert info["lambda"] == lam_o
    lp.close()


def test_lp_every_variable_fixed():
    """All variables fixed: no capacity, so the LP is feasible only for a zero
    budget (s = 0); otherwise the artificial problem, also s = 0."""
    need_gpu()
    from paper_2311_05595_amd import api
    n = 513
    g, a, x, _, delta = _instance(n, 21)
    fixed = np.ones(n, dtype=np.uint8)
    lp = api.LP(n)
    for b in (0.0, 0.3):
        s, info = lp.solve(g, a, x, b, delta, fixed=fixed)
        s_o, _, ok_o = slp.lp_step(g, a, x, b, delta, fixed=fixed)
        assert info["feasible"] == ok_o == (b == 0.0)
        assert np.all(s == 0.0) and np.all(s_o == 0.0)
    lp.close()
