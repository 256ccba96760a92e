"""End-to-end parity of the MGCG solve, compliance and sensitivity against the
oracle's direct solve, plus the solver's edge cases and failure statuses."""

import numpy as np
import pytest

from helpers import MAT, Case, need_gpu, rel

pytestmark = pytest.mark.gpu

# Tolerances of the acceptance bar: displacement <= 1e-8 (relative 2-norm),
# compliance <= 1e-9 (relative); the solves run to a 1e-10 relative residual.
U_TOL, C_TOL, DC_TOL = 1e-8, 1e-9, 1e-8

SOLVE_CASES = [
    ("cantilever", (24, 12, 12), 1, 1, 3, 1, "uniform", "fp64"),  # the 24x12x12 workload
    ("mbb", (16, 8, 8), 1, 1, 3, 2, "grf", "fp64"),
    ("torsion", (12, 6, 6), 1, 2, 2, 3, "grf", "fp64"),
    ("cantilever", (16, 8, 8), 1, 4, 3, 1, "grf", "mixed"),
    ("cantilever", (8, 4, 4), 2, 2, 3, 2, "grf", "mixed"),
    ("mbb", (8, 4, 4), 2, 1, 2, 1, "grf", "fp64"),
    ("cantilever", (10, 6, 6), 1, 1, 1, 1, "grf", "fp64"),        # single level: dense solve
    ("cantilever", (6, 2, 2), 1, 1, 2, 4, "uniform", "mixed"),    # four load cases, ragged
    ("torsion", (16, 8, 8), 1, 1, 4, 4, "uniform", "fp64"),
    # triquadratic elements with three and four load cases in one solve
    ("cantilever", (6, 4, 4), 2, 2, 3, 3, "grf", "mixed"),
    ("torsion", (4, 2, 2), 2, 1, 2, 4, "uniform", "fp64"),
    # 4^3 sub-elements of a triquadratic element (the packed sensitivity
    # contraction), two load cases, ragged element blocks
    ("cantilever", (6, 2, 2), 2, 4, 2, 2, "grf", "fp64"),
    ("mbb", (4, 2, 2), 2, 4, 2, 1, "grf", "mixed"),
    ("cantilever", (4, 2, 2), 2, 4, 2, 3, "grf", "fp64"),
    # bilinear elements with 4^3 sub-elements and four load cases, 30
    # elements (a ragged last block of the contraction)
    ("torsion", (5, 3, 2), 1, 4, 1, 4, "grf", "fp64"),
]


def _id(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-q{c[2]}-n{c[3]}-L{c[4]}-r{c[5]}-{c[6]}-{c[7]}"


@pytest.mark.parametrize("cfg", SOLVE_CASES, ids=_id)
def test_solve_matches_direct(cfg):
    need_gpu()
    kind, nel, order, nsub, nlev, nrhs, field, prec = cfg
    c = Case(kind, nel, order, nsub, nlev, nrhs, field=field, seed=21, precision=prec)
    p = c.problem()
    p.set_densities(c.rho)
    info = p.solve(rtol=1e-10, maxit=3000, warm_start=False)
    assert info["status"] == 0
    for l in range(nrhs):
        assert info["rel_res"][l] <= 1e-10
    u = p.displacement()
    ud = c.direct()
    for l in range(nrhs):
        assert rel(u[l], ud[l]) <= U_TOL, l
        assert np.all(u[l][c.mask.astype(bool)] == 0.0)
    cc, dc = p.compliance_sensitivity()
    cref = c.compliance(ud)
    assert np.all(np.abs(cc[:nrhs] - cref) <= C_TOL * np.abs(cref))
    assert abs(cc[nrhs] - cref.sum()) <= C_TOL * abs(cref.sum())
    dref = c.sensitivity(ud)
    assert rel(dc, dref) <= DC_TOL
    p.close()


def test_warm_start_and_state_reuse():
    need_gpu()
    c = Case("cantilever", (16, 8, 8), 1, 1, 3, 1, seed=5)
    p = c.problem()
    p.set_densities(c.rho)
    i0 = p.solve(rtol=1e-10, warm_start=False)
    u0 = p.displacement().copy()
    i1 = p.solve(rtol=1e-10, warm_start=True)  # from the converged solution
    assert i1["iters"][0] <= 1
    assert rel(p.displacement(), u0) <= 1e-10
    # a perturbed design: warm and cold starts reach the same solution (a
    # warm start need not be faster when void moduli change by decades)
    import workloads as W
    rho2 = W.perturb(c.rho, 99, amp=0.02)
    p.set_densities(rho2)
    iw = p.solve(rtol=1e-10, warm_start=True)
    uw = p.displacement().copy()
    ic = p.solve(rtol=1e-10, warm_start=False)
    assert iw["status"] == 0 and ic["status"] == 0
    assert rel(uw, p.displacement()) <= 1e-7
    # initial guess round trip
    p.set_initial_guess(u0)
    np.testing.assert_array_equal(p.displacement(), u0)
    assert i0["iters"][0] > 0
    p.close()


def test_failure_statuses():
    need_gpu()
    from paper_2311_05595_amd._abi import MGCGError, MGCG_EINVAL, MGCG_ESTATE, MGCG_ENOTCONV
    c = Case("cantilever", (8, 4, 4), 1, 1, 2, 1, seed=1)
    p = c.problem()
    with pytest.raises(MGCGError) as e:
        p.solve()
    assert e.value.code == MGCG_ESTATE
    bad = c.rho.copy()
    bad.flat[7] = np.nan
    with pytest.raises(MGCGError) as e:
        p.set_densities(bad)
    assert e.value.code == MGCG_EINVAL
    bad = c.rho.copy()
    bad.flat[3] = 1.5
    with pytest.raises(MGCGError) as e:
        p.set_densities(bad)
    assert e.value.code == MGCG_EINVAL
    p.set_densities(c.rho)
    info = p.solve(rtol=1e-12, maxit=1, warm_start=False, allow_notconv=True)
    assert info["status"] == MGCG_ENOTCONV and info["iters"][0] == 1
    p.close()


def test_zero_load_and_unsupported_body():
    need_gpu()
    import workloads as W
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError, MGCG_EBREAKDOWN
    nel = (4, 2, 2)
    mask, f = W.make_problem("cantilever", *nel, 1, 2)
    f[1] = 0.0
    rho = W.uniform_field((2, 2, 4), 3, 0.2, 1.0)
    p = api.Problem(nel, mask, f, nlevels=2)
    p.set_densities(rho)
    info = p.solve(rtol=1e-10, warm_start=False)
    assert info["iters"][1] == 0 and np.all(p.displacement()[1] == 0.0)
    p.close()
    # no supports: K is singular (six rigid modes); the coarsest Cholesky or
    # the CG recurrence must report a breakdown instead of returning garbage
    free = np.zeros_like(mask)
    p = api.Problem(nel, free, f, nlevels=2)
    with pytest.raises(MGCGError) as e:
        p.set_densities(rho)
        p.solve(rtol=1e-10, warm_start=False)
    assert e.value.code == MGCG_EBREAKDOWN
    p.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replay_equals_eager_launches(prec):
    """The captured PCG iteration replayed as a HIP graph gives bit-identical
    iterates to launching the same kernels one by one, over several solves
    with the library's own eager work (operator refreshes, warm starts, host
    reads) between the replays."""
    need_gpu()
    import workloads as W
    c = Case("cantilever", (16, 8, 8), 1, 1, 3, 2, seed=31, precision=prec)
    fields = [c.rho, W.perturb(c.rho, 311), W.perturb(c.rho, 312)]
    runs = []
    for mode in ("eager", "graph"):
        p = c.problem()
        p.set_launch_mode(mode)
        out = []
        for j, rho in enumerate(fields):
            p.set_densities(rho)
            info = p.solve(rtol=1e-10, maxit=3000, warm_start=j > 0)
            assert info["status"] == 0
            out.append((info["iters"][:2], p.displacement().copy(),
                        p.compliance_sensitivity(want_dc=False)[0].copy()))
        p.close()
        runs.append(out)
    for (ie, ue, ce), (ig, ug, cg) in zip(*runs):
        assert ie == ig
        assert np.array_equal(ue, ug)
        assert np.array_equal(ce, cg)
    ud = c.direct()
    assert rel(runs[1][0][1][0], ud[0]) <= U_TOL


def test_scaled_warm_start():
    """The scaled warm start multiplies the previous u by the energy
    minimiser f.u / u^T K u: from 2 u* (u* converged) it lands on u* and
    stops at once, where the plain warm start iterates; from a converged u*
    it is the plain warm start.  Both reach the direct solve."""
    need_gpu()
    c = Case("cantilever", (16, 8, 8), 1, 1, 3, 2, seed=41)
    p = c.problem()
    p.set_densities(c.rho)
    assert p.solve(rtol=1e-10, maxit=3000, warm_start="cold")["status"] == 0
    u = p.displacement().copy()
    p.set_initial_guess(2.0 * u)
    i_scaled = p.solve(rtol=2e-10, maxit=3000, warm_start="scaled")
    assert max(i_scaled["iters"][:2]) <= 1
    p.set_initial_guess(2.0 * u)
    i_plain = p.solve(rtol=2e-10, maxit=3000, warm_start="plain")
    assert min(i_plain["iters"][:2]) >= 5
    ud = c.direct()
    for l in range(2):
        assert rel(p.displacement()[l], ud[l]) <= U_TOL
    # a zero guess: the factor is 0 (x^T K x = 0), a cold start
    p.set_initial_guess(np.zeros_like(u))
    i0 = p.solve(rtol=1e-10, maxit=3000, warm_start="scaled")
    assert i0["status"] == 0 and rel(p.displacement()[0], ud[0]) <= U_TOL
    p.close()


@pytest.mark.parametrize("field,order,nsub", [("void", 1, 1), ("binary", 1, 2), ("binary", 2, 1)])
def test_densities_at_their_bounds(field, order, nsub):
    """Densities exactly 0 and 1: an all-void body (every modulus E_min, the
    operator 1e-9 of the solid one) and a random 0/1 design; u and c against
    the oracle's direct solve."""
    need_gpu()
    c = Case("cantilever", (6, 4, 4), order, nsub, 2, 1, seed=71)
    if field == "void":
        c.rho = np.zeros_like(c.rho)
    else:
        c.rho = (np.random.default_rng(72).uniform(size=c.rho.shape) < 0.5).astype(np.float64)
    p = c.problem()
    p.set_densities(c.rho)
    info = p.solve(rtol=1e-10, maxit=3000, warm_start=False)
    assert info["status"] == 0
    u = p.displacement()
    cc, _ = p.compliance_sensitivity(want_dc=False)
    p.close()
    ud = c.direct()
    assert rel(u[0], ud[0]) <= U_TOL
    cref = c.compliance(ud)
    assert abs(cc[0] - cref[0]) <= C_TOL * abs(cref[0])
