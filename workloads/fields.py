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
* ``solid_at_supports_and_loads``: density 1 in every Q1 element that touches
  a fixed or loaded node, the non-design solid layer of the paper's bridge
  (Sec. 7.1) applied to every support and load.  A random field alone can
  leave a load or a support in void; the displacement there then grows like
  1/Emin and the FP64 residual ||f - K u|| cannot fall below roughly
  eps |K| |u|, far above 1e-8 of ||f||.
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


def solid_at_supports_and_loads(rho, mask, f, nel, nsub):
    """Copy of ``rho`` (lattice ``(nsub*nelz, nsub*nely, nsub*nelx)``) with
    every sub-density of a Q1 element set to 1 when one of the element's 8
    nodes has a fixed DOF (``mask``) or a nonzero load in any load case
    (``f``, ``[load case][DOF]``)."""
    nx, ny, nz = nel
    touched = np.asarray(mask, dtype=bool).reshape(-1, 3).any(axis=1)
    touched |= (np.atleast_2d(f) != 0.0).reshape(np.atleast_2d(f).shape[0], -1, 3).any(axis=(0, 2))
    t = touched.reshape(nz + 1, ny + 1, nx + 1)
    el = np.zeros((nz, ny, nx), dtype=bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                el |= t[dz:dz + nz, dy:dy + ny, dx:dx + nx]
    sub = np.repeat(np.repeat(np.repeat(el, nsub, axis=0), nsub, axis=1), nsub, axis=2)
    out = np.array(rho, dtype=np.float64, copy=True).reshape(sub.shape)
    out[sub] = 1.0
    return out
