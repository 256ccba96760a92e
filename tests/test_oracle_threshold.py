"""Pins of the oracle's thresholding (Sec. 5): the density-value rule, the
angle condition and the Heaviside projection with its volume-preserving
threshold."""

import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import threshold as T


def test_pre_round():
    r = T.pre_round([0.0, 0.04, 0.05, 0.0500001, 0.5, 0.9499999, 0.95, 0.99, 1.0])
    assert list(r) == [0.0, 0.0, 0.0, 0.0500001, 0.5, 0.9499999, 1.0, 1.0, 1.0]


@pytest.mark.parametrize("n,vfrac,seed", [(10, 0.3, 0), (97, 0.5, 1), (300, 0.25, 2)])
def test_density_threshold_brute_force(n, vfrac, seed):
    rng = np.random.default_rng(seed)
    rho = np.round(rng.random(n), 2)  # many equal values
    out = T.density_threshold(rho, vfrac)
    k = int(math.floor(vfrac * n))
    assert out.sum() == k and set(np.unique(out)) <= {0.0, 1.0}
    ones, zeros = np.flatnonzero(out == 1.0), np.flatnonzero(out == 0.0)
    for i in ones:
        for j in zeros:
            # nothing left at 0 is above something set to 1; equal values in index order
            assert rho[j] < rho[i] or (rho[j] == rho[i] and j > i)


def test_angle_condition():
    g = np.array([1.0, 0.0])
    for deg in (10.0, 60.0, 89.8, 89.95, 120.0):
        th = math.radians(deg)
        d = -np.array([math.cos(th), math.sin(th)])  # angle deg between -g and d
        assert T.angle_cos(g, d) == pytest.approx(math.cos(th), abs=1e-15)
        assert T.angle_ok(g, d) == (deg < 89.9)


def test_heaviside_closed_forms():
    for beta in (1.0, 8.0, 64.0):
        for eta in (0.2, 0.5, 0.8):
            h = T.heaviside([0.0, 1.0, eta], beta, eta)
            assert h[0] == pytest.approx(0.0, abs=1e-15)
            assert h[1] == pytest.approx(1.0, rel=1e-15)
            assert h[2] == pytest.approx(
                math.tanh(beta * eta) / (math.tanh(beta * eta) + math.tanh(beta * (1 - eta))),
                rel=1e-15)
    # h(rho, beta, 0) >= rho and h(rho, beta, 1) <= rho (Sec. 5.4)
    rho = np.linspace(0.0, 1.0, 101)
    assert np.all(T.heaviside(rho, 4.0, 1e-9) >= rho - 1e-12)
    assert np.all(T.heaviside(rho, 4.0, 1.0 - 1e-9) <= rho + 1e-12)


@pytest.mark.parametrize("beta,seed", [(1.0, 0), (2.0, 1), (16.0, 2), (100.0, 3)])
def test_eta_newton_against_brentq(beta, seed):
    rng = np.random.default_rng(seed)
    rho = np.clip(rng.beta(0.7, 1.2, 5000), 0.0, 1.0)
    eta = T.eta_newton(rho, beta)
    ref = brentq(lambda e: T.volume_gap(rho, beta, e), 1e-12, 1.0 - 1e-12, xtol=1e-15)
    assert abs(eta - ref) <= 1e-10
    # the projection keeps the volume
    assert abs(T.heaviside(rho, beta, eta).sum() - rho.sum()) <= 1e-9 * rho.sum()


def test_eta_derivative_matches_differences():
    rng = np.random.default_rng(4)
    rho = rng.random(200)
    for beta, eta in [(2.0, 0.3), (10.0, 0.6)]:
        h = 1e-6
        fd = (T.volume_gap(rho, beta, eta + h) - T.volume_gap(rho, beta, eta - h)) / (2 * h)
        assert T.volume_gap_derivative(rho, beta, eta) == pytest.approx(fd, rel=1e-6)


def test_lagrangian_strategy_hand_case():
    """rho = (0.2, 0.5, 0.8), g = (-1, 1, -1): alpha = (0.8, 0.5, 0.2).  The
    first density may not reach 1 (0.2 < v_u), so alpha~ < 0.8; at 0.5 the
    step is d = (0.5, -0.5, 0.2) with cosine 1.2 / (sqrt(3) sqrt(0.54)) > 0:
    alpha~ = 0.5, rho~ = (0.7, 0, 1)."""
    rho_t, a = T.lagrangian_threshold([0.2, 0.5, 0.8], [-1.0, 1.0, -1.0])
    assert a == 0.5
    assert np.allclose(rho_t, [0.7, 0.0, 1.0], rtol=0, atol=1e-15)
    assert T.angle_cos([-1.0, 1.0, -1.0], rho_t - [0.2, 0.5, 0.8]) == pytest.approx(
        1.2 / (math.sqrt(3.0) * math.sqrt(0.54)), rel=1e-14)


@pytest.mark.parametrize("m,binds", [(3000, False), (6000, True)])
def test_lagrangian_strategy_angle_binds(m, binds):
    """One density with a large gradient (rho = 0.94, g = -1e3, alpha = 6e-5)
    and m with tiny ones (rho = 0.5, g = +-1e-6, alpha = 5e5).  At alpha = 5e5
    the step is 0.06 on the first and 0.5 on the others:
    cos = (1e6 * 6e-5 + m * 1e-12 * 5e5) / (|g| sqrt(0.0036 + 0.25 m)),
    0.00219 for m = 3000 (passes 89.9 degrees, cos = 0.001745) and 0.00155
    for m = 6000 (fails): alpha~ falls back to 6e-5."""
    rho = np.full(m + 1, 0.5)
    g = np.where(np.arange(m + 1) % 2 == 0, 1e-6, -1e-6)
    rho[0], g[0] = 0.94, -1e3
    c = (1e6 * 6e-5 + m * 1e-12 * 5e5) / (math.sqrt(1e6 + m * 1e-12) * math.sqrt(0.0036 + 0.25 * m))
    assert (c <= math.cos(math.radians(89.9))) == binds
    rho_t, a = T.lagrangian_threshold(rho, g)
    if binds:
        assert a == pytest.approx(6e-5, rel=1e-12)
        assert rho_t[0] == 1.0 and np.all(np.abs(rho_t[1:] - 0.5) < 1e-9)
    else:
        assert a == pytest.approx(5e5, rel=1e-12)
        assert rho_t[0] == 1.0 and np.all(rho_t[1:] == np.where(g[1:] > 0, 0.0, 1.0))


def _closed_form_choice(rho, g, v_u=0.3, v_l=0.7):
    """alpha~ from cos(alpha) = sum g^2 m / (|g| sqrt(sum g^2 m^2)) with
    m_i = min(alpha, alpha_i): the largest candidate below the first
    safeguard violation whose cosine passes."""
    alpha = T.lagrangian_alphas(rho, g)
    bad = ((g < 0) & (rho < v_u)) | ((g > 0) & (rho > v_l))
    viol = alpha[bad].min() if bad.any() else np.inf
    w = g * g
    cmax = math.cos(math.radians(89.9))
    cands = np.unique(alpha[np.isfinite(alpha) & (alpha > 0) & (alpha < viol)])
    cos = np.array([np.sum(w * np.minimum(a, alpha)) /
                    (math.sqrt(w.sum()) * math.sqrt(np.sum(w * np.minimum(a, alpha) ** 2)))
                    for a in cands])
    ok = cands[cos > cmax]
    return (ok.max() if ok.size else 0.0), cos


@pytest.mark.parametrize("seed", range(6))
def test_lagrangian_strategy_matches_closed_form(seed):
    rng = np.random.default_rng(seed)
    n = 400
    rho = T.pre_round(rng.beta(0.6, 0.6, n))
    g = rng.standard_normal(n) * rng.exponential(1.0, n) ** 3
    g[rng.random(n) < 0.05] = 0.0
    if seed % 2:
        g[rng.random(n) < 0.5] *= 1e-4  # the angle condition matters
    rho_t, a = T.lagrangian_threshold(rho, g)
    ref, cos = _closed_form_choice(rho, g)
    assert a == ref
    # the cosine is nonincreasing in alpha
    assert np.all(np.diff(cos) <= 1e-12)
    # the safeguards hold at alpha~ and rho~ lies in the box
    moved = (T.lagrangian_alphas(rho, g) <= a) & (g != 0)
    assert np.all(rho[moved & (g < 0)] >= 0.3) and np.all(rho[moved & (g > 0)] <= 0.7)
    assert np.all((rho_t >= 0) & (rho_t <= 1))
    assert np.all(rho_t[moved & (g > 0)] == 0.0) and np.all(rho_t[moved & (g < 0)] == 1.0)
