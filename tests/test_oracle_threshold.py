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
