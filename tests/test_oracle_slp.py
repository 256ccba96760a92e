"""Pins of the oracle's SLP step (Sec. 4): the LP subproblem (Pstar) against an
enumeration of the polytope's vertices and against scipy's linprog, its KKT
conditions, and the step-control rules of Algorithm 2 on hand-computed cases."""

import itertools

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import slp


def _instance(n, seed, delta=0.2, budget=0.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    g = -rng.exponential(1.0, n) + 0.2 * rng.standard_normal(n)
    a = rng.uniform(0.5, 1.5, n)
    return g, a, x, budget, delta


def _vertices_min(g, a, l, u, b):
    """Minimum of g^T s over the vertices of {a^T s = b, l <= s <= u}: every
    vertex has at most one coordinate strictly inside its bounds."""
    n = g.size
    best = np.inf
    for k in range(-1, n):
        others = [i for i in range(n) if i != k]
        for bits in itertools.product((0, 1), repeat=len(others)):
            s = np.empty(n)
            for i, bt in zip(others, bits):
                s[i] = u[i] if bt else l[i]
            if k >= 0:
                s[k] = (b - sum(a[i] * s[i] for i in others)) / a[k]
                if s[k] < l[k] - 1e-12 or s[k] > u[k] + 1e-12:
                    continue
            elif abs(a @ s - b) > 1e-12:
                continue
            best = min(best, g @ s)
    return best


@pytest.mark.parametrize("n,seed,b", [(1, 0, 0.0), (4, 1, 0.0), (6, 2, 0.05), (8, 3, -0.05),
                                      (9, 4, 0.1)])
def test_lp_against_vertex_enumeration(n, seed, b):
    g, a, x, _, delta = _instance(n, seed)
    l, u = slp.lp_bounds(x, delta)
    if not (a @ l <= b <= a @ u):
        b = 0.5 * (a @ l + a @ u)
    s, lam, ok = slp.lp_step(g, a, x, b, delta)
    assert ok
    assert np.all(s >= l - 1e-15) and np.all(s <= u + 1e-15)
    assert abs(a @ s - b) <= 1e-12
    assert abs(g @ s - _vertices_min(g, a, l, u, b)) <= 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_lp_against_linprog_and_kkt(seed):
    n = 300
    g, a, x, _, delta = _instance(n, 10 + seed, delta=0.1)
    l, u = slp.lp_bounds(x, delta)
    b = (a @ l) + 0.37 * (a @ (u - l))
    s, lam, ok = slp.lp_step(g, a, x, b, delta)
    ref = linprog(g, A_eq=a[None, :], b_eq=[b], bounds=list(zip(l, u)), method="highs")
    assert ref.status == 0
    assert abs(g @ s - ref.fun) <= 1e-9 * abs(ref.fun)
    # without ties the minimiser is unique
    assert np.abs(s - ref.x).max() <= 1e-9
    # KKT: the Lagrangian g + lambda a is <= 0 where s = u, >= 0 where s = l
    rc = g + lam * a
    at_u, at_l = s >= u - 1e-14, s <= l + 1e-14
    assert np.all(rc[at_u & ~at_l] <= 1e-12)
    assert np.all(rc[at_l & ~at_u] >= -1e-12)
    assert (~at_u & ~at_l).sum() <= 1


def test_lp_ties_take_index_order():
    """Equal ratios: the budget goes to the lower indices first; the optimum
    value is the same for any split."""
    n = 6
    g = np.full(n, -1.0)
    a = np.ones(n)
    x = np.full(n, 0.5)
    s, lam, ok = slp.lp_step(g, a, x, 0.25, 0.1)
    # from s = -0.1 everywhere, budget 0.25 + 0.6 = 0.85 over capacities 0.2
    assert ok and lam == 1.0
    assert np.allclose(s, [0.1, 0.1, 0.1, 0.1, -0.1 + 0.05, -0.1])


def test_lp_infeasible_uses_shrunk_box():
    g, a, x, _, delta = _instance(5, 7, delta=0.1)
    l, u = slp.lp_bounds(x, delta)
    s, lam, ok = slp.lp_step(g, a, x, a @ l - 1.0, delta)
    assert not ok and np.allclose(s, slp.lp_bounds(x, 0.08)[0])
    s, lam, ok = slp.lp_step(g, a, x, a @ u + 1.0, delta)
    assert not ok and np.allclose(s, slp.lp_bounds(x, 0.08)[1])


def test_theta_and_trust_rules():
    # eq. (theta2): P_opt <= P_fsb / 2 gives 0.5 P_fsb / (P_fsb - P_opt)
    assert slp.theta_update(0, [1.0], 1.0, 2.0, -1.0) == pytest.approx(1.0 / 3.0)
    # otherwise theta_sup = 1 and theta_large = (1 + N / 1) min(history) caps nothing
    assert slp.theta_update(0, [1.0], 1.0, 2.0, 1.5) == 1.0
    assert slp.theta_update(3, [1.0, 0.2], 0.5, 2.0, 1.5) == 0.5
    # theta_large: (1 + N / (k + 1)^1.1) min(history) with a small N
    assert slp.theta_update(1, [0.4, 0.3], 1.0, 2.0, 1.5, N=1.0) == pytest.approx(
        (1 + 1 / 2 ** 1.1) * 0.3)
    # reject: delta = min(0.25 |s|_inf, 0.1 delta)
    assert slp.trust_update(0.05, 1.0, 0.2, 0.2, 1.0, 1e-3) == (False, pytest.approx(0.02))
    # accept, good: min(2 delta, box) then max(., delta_min)
    assert slp.trust_update(0.6, 1.0, 0.2, 0.2, 1.0, 1e-3) == (True, pytest.approx(0.4))
    assert slp.trust_update(0.6, 1.0, 0.7, 0.2, 1.0, 1e-3) == (True, pytest.approx(1.0))
    # accept, modest: unchanged but at least delta_min
    assert slp.trust_update(0.2, 1.0, 1e-4, 1e-4, 1.0, 1e-3) == (True, pytest.approx(1e-3))


def test_merit_reductions_identities():
    """With c = 0 before and after, A_red = theta (f0 - f1) and
    P_red = -theta g^T s - (1 - theta) (a^T s)^2 / 2."""
    g, a, x, _, delta = _instance(7, 9)
    s = np.random.default_rng(1).uniform(-delta, delta, 7)
    ar, pr, pf, po = slp.merit_reductions(0.3, 2.0, 1.5, g, s, 0.0, 0.0, a)
    assert ar == pytest.approx(0.3 * 0.5)
    assert pr == pytest.approx(-0.3 * (g @ s) - 0.7 * 0.5 * (a @ s) ** 2)
    assert pf == pytest.approx(-0.5 * (a @ s) ** 2) and po == pytest.approx(-(g @ s))
    # theta_sup is the largest theta with P_red >= P_fsb / 2
    for pf_, po_ in [(2.0, 0.5), (1.0, -3.0), (0.5, 0.1)]:
        th = slp.theta_update(0, [1.0], 1.0, pf_, po_)
        if th < 1.0:
            assert th * po_ + (1 - th) * pf_ == pytest.approx(0.5 * pf_)


@pytest.mark.parametrize("seed", range(3))
def test_lp_fixed_variables_against_linprog(seed):
    """Fixed variables (Sec. 6.1) held at zero: the same optimum as linprog
    with the bounds (0, 0) for them, and s = 0 there."""
    n = 200
    g, a, x, _, delta = _instance(n, 20 + seed, delta=0.1)
    fixed = (np.random.default_rng(seed).random(n) < 0.3).astype(np.uint8)
    l, u = slp.lp_bounds(x, delta, fixed=fixed)
    assert np.all(l[fixed == 1] == 0.0) and np.all(u[fixed == 1] == 0.0)
    b = (a @ l) + 0.41 * (a @ (u - l))
    s, lam, ok = slp.lp_step(g, a, x, b, delta, fixed=fixed)
    ref = linprog(g, A_eq=a[None, :], b_eq=[b], bounds=list(zip(l, u)), method="highs")
    assert ok and ref.status == 0
    assert abs(g @ s - ref.fun) <= 1e-9 * abs(ref.fun)
    assert np.all(s[fixed == 1] == 0.0)
