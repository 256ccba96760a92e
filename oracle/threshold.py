"""Density thresholding of Sec. 5 (plain definitions).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Rounding of the densities very close to 0 or 1 (Sec. 5: rho >= 0.95 -> 1,
  rho <= 0.05 -> 0).
* The strategy based on the density values (Sec. 5.1): with the densities in
  descending order, the floor(v_frac n) highest are set to 1 and the rest to
  0.  Reading: equal densities are taken in increasing index order.
* The angle condition (eq. (angle)): -gL^T d / (|gL| |d|) > cos(theta_max),
  theta_max = 89.9 degrees.
* The strategy based on the gradient of the Lagrangian (Sec. 5.2): with
  g = grad L, alpha_i is the step at which rho_i - alpha g_i reaches 0
  (g_i > 0: alpha_i = rho_i / g_i) or 1 (g_i < 0: alpha_i = (1 - rho_i) / -g_i);
  rho~(alpha) is rho - alpha g projected onto [0, 1], and alpha~ is the
  largest alpha_i at which rho~ keeps the safeguards (a density may reach 1
  only if rho_i >= v_u = 0.3, reach 0 only if rho_i <= v_l = 0.7) and
  satisfies the angle condition with d = rho~ - rho.  Readings: the
  safeguards test the density before the step (the densities are the
  pre-rounded ones); a component with alpha_i <= alpha is set to its bound
  exactly (the projection in exact arithmetic), the others take
  rho_i - alpha g_i; components with g_i = 0 never move; alpha_i = 0 (a density
  already at the bound it would reach) is no candidate, since d = 0 there
  for it; with no admissible candidate alpha~ = 0 and rho~ = rho.
* The smooth Heaviside projection of Sec. 5.4,
      h(rho, beta, eta) = (tanh(beta eta) + tanh(beta (rho - eta)))
                          / (tanh(beta eta) + tanh(beta (1 - eta))),
  with eta the zero of f(eta) = sum_i v_i h(rho_i, beta, eta) - sum_i v_i rho_i
  found by Newton's method.  Readings: the cells of a lattice have equal
  volumes, so v cancels; Newton starts from eta = 1/2, keeps the bracket
  [lo, hi] of the sign change (f(0) > 0 > f(1), Sec. 5.4), takes the midpoint
  of the bracket when a Newton step leaves it, and stops when |delta eta| <=
  1e-14 or |f| <= 1e-13 sum_i rho_i, at most 100 iterations.

Pins (tests/test_oracle_threshold.py): the gradient strategy on a
hand-computed three-density case, on a case built so that the angle
condition binds, and against the same choice made from closed-form sums
(cos(alpha) = sum g^2 m / (|g| sqrt(sum g^2 m^2)), m_i = min(alpha, alpha_i), a
nonincreasing function of alpha); the top-k rule against a brute-force
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


def lagrangian_alphas(rho, gL):
    """alpha_i of Sec. 5.2 (inf where g_i = 0)."""
    rho = np.asarray(rho, dtype=np.float64)
    g = np.asarray(gL, dtype=np.float64)
    alpha = np.full(rho.shape, np.inf)
    pos, neg = g > 0.0, g < 0.0
    alpha[pos] = rho[pos] / g[pos]
    alpha[neg] = (1.0 - rho[neg]) / -g[neg]
    return alpha


def lagrangian_step(rho, gL, alpha_t):
    """rho~ at the step alpha_t: bounds for alpha_i <= alpha_t, else rho - alpha_t g."""
    rho = np.asarray(rho, dtype=np.float64)
    g = np.asarray(gL, dtype=np.float64)
    alpha = lagrangian_alphas(rho, g)
    out = rho - alpha_t * g
    hit = (alpha <= alpha_t) & (g != 0.0)
    out[hit & (g > 0.0)] = 0.0
    out[hit & (g < 0.0)] = 1.0
    return np.clip(out, 0.0, 1.0)


def lagrangian_threshold(rho, gL, v_u=0.3, v_l=0.7, theta_max_deg=89.9):
    """(rho~, alpha~) of the strategy based on the gradient of the Lagrangian:
    every candidate alpha_i > 0 is tried, in ascending order."""
    rho = np.asarray(rho, dtype=np.float64)
    g = np.asarray(gL, dtype=np.float64)
    alpha = lagrangian_alphas(rho, g)
    # a density rounded to 1 needs rho_i >= v_u, one rounded to 0 rho_i <= v_l
    bad = ((g < 0.0) & (rho < v_u)) | ((g > 0.0) & (rho > v_l))
    best = 0.0
    for a in sorted(set(alpha[np.isfinite(alpha) & (alpha > 0.0)].tolist())):
        if np.any(bad & (alpha <= a)):
            break  # every larger alpha rounds this density too
        if angle_ok(g, lagrangian_step(rho, g, a) - rho, theta_max_deg):
            best = a
    if best == 0.0:
        return rho.copy(), 0.0
    return lagrangian_step(rho, g, best), best


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


__all__ = ["pre_round", "density_threshold", "angle_cos", "angle_ok", "lagrangian_alphas",
           "lagrangian_step", "lagrangian_threshold", "heaviside",
           "volume_gap", "volume_gap_derivative", "eta_newton"]
