"""Density thresholding of Sec. 5 (plain definitions).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Rounding of the densities very close to 0 or 1 (Sec. 5: rho >= 0.95 -> 1,
  rho <= 0.05 -> 0).
* The strategy based on the density values (Sec. 5.1): with the densities in
  descending order, the floor(v_frac n) highest are set to 1 and the rest to
  0.  Reading: equal densities are taken in increasing index order.
* The angle condition (eq. (angle)): -gL^T d / (|gL| |d|) > cos(theta_max),
  theta_max = 89.9 degrees.
* The smooth Heaviside projection of Sec. 5.4,
      h(rho, beta, eta) = (tanh(beta eta) + tanh(beta (rho - eta)))
                          / (tanh(beta eta) + tanh(beta (1 - eta))),
  with eta the zero of f(eta) = sum_i v_i h(rho_i, beta, eta) - sum_i v_i rho_i
  found by Newton's method.  Readings: the cells of a lattice have equal
  volumes, so v cancels; Newton starts from eta = 1/2, keeps the bracket
  [lo, hi] of the sign change (f(0) > 0 > f(1), Sec. 5.4), takes the midpoint
  of the bracket when a Newton step leaves it, and stops when |delta eta| <=
  1e-14 or |f| <= 1e-13 sum_i rho_i, at most 100 iterations.

Pins (tests/test_oracle_threshold.py): the top-k rule against a brute-force
check of every pair (no density set to 0 exceeds one set to 1, ties in index
order) and its exact count; h at closed-form points (h(0) = 0, h(1) = 1,
h(eta) = tanh(beta eta) / (tanh(beta eta) + tanh(beta (1 - eta)))); eta against
scipy's brentq root of the same f; the volume preserved; the angle test on
vectors at known angles.
"""

import math

import numpy as np


def pre_round(rho, lo=0.05, hi=0.95):
    rho = np.array(rho, dtype=np.float64)
    rho[rho >= hi] = 1.0
    rho[rho <= lo] = 0.0
    return rho


def density_threshold(rho, vfrac):
    """floor(vfrac n) highest densities to 1, the rest to 0 (ties in index order)."""
    rho = np.asarray(rho, dtype=np.float64)
    k = int(math.floor(vfrac * rho.size))
    order = sorted(range(rho.size), key=lambda i: (-rho[i], i))
    out = np.zeros_like(rho)
    out[order[:k]] = 1.0
    return out


def angle_cos(gL, d):
    """-gL^T d / (|gL| |d|)."""
    gL = np.asarray(gL, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    return -float(gL @ d) / (float(np.linalg.norm(gL)) * float(np.linalg.norm(d)))


def angle_ok(gL, d, theta_max_deg=89.9):
    return angle_cos(gL, d) > math.cos(math.radians(theta_max_deg))


def heaviside(rho, beta, eta):
    rho = np.asarray(rho, dtype=np.float64)
    num = math.tanh(beta * eta) + np.tanh(beta * (rho - eta))
    den = math.tanh(beta * eta) + math.tanh(beta * (1.0 - eta))
    return num / den


def volume_gap(rho, beta, eta):
    """f(eta) of Sec. 5.4 with equal cell volumes (v = 1)."""
    return float(np.sum(heaviside(rho, beta, eta))) - float(np.sum(rho))


def volume_gap_derivative(rho, beta, eta):
    """d f / d eta."""
    rho = np.asarray(rho, dtype=np.float64)
    te, t1 = math.tanh(beta * eta), math.tanh(beta * (1.0 - eta))
    tr = np.tanh(beta * (rho - eta))
    num = te + tr
    den = te + t1
    dnum = beta * (1.0 - te * te) - beta * (1.0 - tr * tr)
    dden = beta * (1.0 - te * te) - beta * (1.0 - t1 * t1)
    return float(np.sum((dnum * den - num * dden) / (den * den)))


def eta_newton(rho, beta, max_iter=100):
    """eta with f(eta) = 0 by Newton's method with a bisection safeguard."""
    s = float(np.sum(rho))
    lo, hi, eta = 0.0, 1.0, 0.5
    for _ in range(max_iter):
        f = volume_gap(rho, beta, eta)
        if abs(f) <= 1e-13 * s:
            break
        if f > 0.0:
            lo = eta
        else:
            hi = eta
        df = volume_gap_derivative(rho, beta, eta)
        nxt = eta - f / df if df != 0.0 else 0.5 * (lo + hi)
        if not (lo < nxt < hi):
            nxt = 0.5 * (lo + hi)
        if abs(nxt - eta) <= 1e-14:
            eta = nxt
            break
        eta = nxt
    return eta


__all__ = ["pre_round", "density_threshold", "angle_cos", "angle_ok", "heaviside",
           "volume_gap", "volume_gap_derivative", "eta_newton"]
