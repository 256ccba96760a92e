"""Seeded density fields.

* ``uniform_field``: i.i.d. uniform densities in ``[lo, hi]``.
* ``gaussian_random_field``: white noise smoothed by a separable Gaussian of
  standard deviation ``corr/2`` lattice cells (reflective boundaries), then
  standardised and squashed by a logistic of slope 1/0.5 onto
  ``[rho_min, 1]``, with the logistic's offset found by bisection so that the
  mean density equals ``volfrac``.  This mimics the smooth, mostly-void,
  0/1-leaning designs of an optimisation run (SIMP designs at volume fraction
  0.2-0.3).
* ``perturb``: an SLP-like step, ``clip(rho + U(-amp, amp), rho_min, 1)``.
"""

import numpy as np
from scipy import ndimage


def uniform_field(shape, seed, lo=0.05, hi=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(np.float64)


def _logistic(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def gaussian_random_field(shape, seed, corr=6.0, rho_min=1e-3, volfrac=0.3):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=shape)
    g = ndimage.gaussian_filter(g, sigma=corr / 2.0, mode="reflect")
    g = (g - g.mean()) / g.std()

    def field(t):
        return rho_min + (1.0 - rho_min) * _logistic((g - t) / 0.5)

    lo, hi = -20.0, 20.0  # mean(field) decreases with t
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if field(mid).mean() > volfrac:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    return field(0.5 * (lo + hi)).astype(np.float64)


def perturb(rho, seed, amp=0.05, rho_min=1e-3):
    rng = np.random.default_rng(seed)
    return np.clip(rho + rng.uniform(-amp, amp, size=rho.shape), rho_min, 1.0)
