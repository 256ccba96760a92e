"""Explicit sparse multigrid components (Sec. 2.3, Algorithm 1).

* Coarse mesh: every coarse element holds 2x2x2 fine elements (Sec. 2.3);
  on the node lattice the coarse node (I, J, K) coincides with the fine node
  (2I, 2J, 2K).  A fine mesh of degree p >= 2 (lattice spacing 1/p)
  coarsens first onto the vertex lattice of the same elements (coarse node
  I on fine node pI), then on as for linear meshes.
* Prolongation P: linear (trilinear) interpolation on the node lattice,
  per displacement component (Sec. 2.3: linear interpolation for Lagrange
  elements; for serendipity elements the paper interpolates with the
  element's shape functions, which on the vertex lattice are the trilinear
  ones); 1-D weights 1 at coincident nodes and, for a fine node q/r of
  the way from coarse node I to I + 1 (ratio r = 2 or 3), 1 - q/r and q/r;
  the 3-D operator is the Kronecker product of the three 1-D ones.
  Restriction R = P^T (Sec. 2.3).
* Supports: a coarse DOF is fixed when its coincident fine DOF is fixed;
  rows of P at fixed fine DOFs and columns at fixed coarse DOFs are zeroed,
  giving P~ = Z_f P Z_c.  Coarse operator (Galerkin):
  A_c = P~^T A_f P~ + (I - Z_c).
* Smoother: weighted Jacobi x <- x + W D^{-1} (b - A x) with per-DOF
  weights w_i = min(omega, theta * A_ii / sum_j |A_ij|), theta = 1.9.  The
  paper tunes one omega experimentally (Sec. 7.2); for rough density fields
  lambda_max(D^{-1} A) exceeds 2/omega at omega = 0.6, the smoother diverges
  on the highest modes and the V-cycle stops being positive definite.  With
  the cap every Gershgorin row sum of W D^{-1} A is at most theta < 2, so the
  smoother is convergent (and the symmetric V-cycle SPD) for any densities;
  omega itself is kept wherever that bound allows it.
* ``vcycle``: Algorithm 1 applied recursively (pre-smoothing from x = 0,
  residual, restriction, coarse solve (exact on the coarsest level),
  prolongation and correction, post-smoothing).  This is the preconditioner
  M as a plain linear map, for testing the HIP V-cycle.
* Smoother on a quadratic or cubic finest level (Sec. 7.5 prefers SSOR
  there): a symmetric Gauss-Seidel in multicolour order.  Nodes of the
  lattice of degree p are coloured by (i mod (p+1), j mod (p+1), k mod
  (p+1)); two nodes of one colour are at least p + 1 lattice steps apart in
  some axis, while an element spans p, so they share no element and their
  rows do not couple.  A forward sweep updates colour 0 .. (p+1)^3 - 1 and,
  within a colour, component x, y, z (each DOF from the latest values,
  relaxation 1); the backward sweep runs colours and components in
  reverse.  Read as one
  forward sweep before and one backward sweep after the coarse correction,
  so the V-cycle stays symmetric.  Coarser (trilinear) levels keep the
  capped Jacobi sweep.
* ``mgcg``: the conjugate gradient method preconditioned by that V-cycle
  (the paper's solver, Sec. 2.3 and 7.2), stopping on
  ||f - K u|| <= rtol ||f||; used where a direct factorisation is too large.

Pins (tests/test_oracle_multigrid.py): P reproduces multilinear fields
exactly, for halving and for the cubic lattice's ratio-3 step (weights 1,
2/3, 1/3); Galerkin of a constant-modulus operator equals the rediscretised
operator with twice the element size (K scales with h in 3-D); the masked
Galerkin operator is symmetric with identity rows on fixed DOFs and positive
definite on free ones; the capped Jacobi sweep has spectral radius < 1 and
the V-cycle is symmetric positive definite even on a rough field where the
plain omega = 0.6 sweep diverges; without smoothing the cycle is the exact
coarse correction, so M A is the A-orthogonal projector onto the range of
the prolongations (idempotent, which fixes the scale of the transfers); with
one sweep before and after, I - M A is the product of the sweep's and the
coarse correction's error propagators; the projector identity holds for a
cubic finest level too (Lagrange and serendipity); mgcg agrees with the
direct solve (linear, quadratic and cubic elements).
The multicolour Gauss-Seidel sweep equals x + (D + L)^-1 (b - A x) (and
the backward one the upper-triangle form) with A ordered by gs_order,
computed by a sparse triangular solve, and its colour classes do not
couple (those of one colour fewer per axis do); the V-cycle with it is
symmetric positive definite and its MG-CG reaches the direct solve, for
quadratic elements in fewer iterations than with the Jacobi sweep.
"""

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla


def prolong_1d(nc, ratio=2):
    """1-D linear interpolation from a lattice of nc nodes to one of
    ratio (nc-1) + 1."""
    nf = ratio * (nc - 1) + 1
    rows, cols, vals = [], [], []
    for I in range(nc):
        rows.append(ratio * I); cols.append(I); vals.append(1.0)
        if I + 1 < nc:
            for q in range(1, ratio):
                rows += [ratio * I + q, ratio * I + q]
                cols += [I, I + 1]
                vals += [1.0 - q / ratio, q / ratio]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def coarse_dims(dims, ratio=2):
    for d in dims:
        if (d - 1) % ratio != 0 or d < ratio + 1:
            raise ValueError(f"lattice {dims} cannot be coarsened by {ratio}")
    return tuple((d - 1) // ratio + 1 for d in dims)


def prolongation(dims_c, ratio=2):
    """DOF prolongation from coarse lattice dims_c (x, y, z) to its
    refinement by `ratio`, unmasked."""
    Px, Py, Pz = (prolong_1d(d, ratio) for d in dims_c)
    Pn = sp.kron(Pz, sp.kron(Py, Px))
    return sp.kron(Pn, sp.identity(3)).tocsr()


def coarse_mask(mask_f, dims_f, ratio=2):
    nx, ny, nz = dims_f
    m = np.asarray(mask_f).reshape(nz, ny, nx, 3)
    return np.ascontiguousarray(m[::ratio, ::ratio, ::ratio, :]).ravel()


def masked_prolongation(dims_c, mask_f, mask_c, ratio=2):
    P = prolongation(dims_c, ratio)
    Zf = sp.diags((np.asarray(mask_f) == 0).astype(np.float64))
    Zc = sp.diags((np.asarray(mask_c) == 0).astype(np.float64))
    return (Zf @ P @ Zc).tocsr()


def galerkin(A_f, Pm, mask_c):
    free_c = (np.asarray(mask_c) == 0).astype(np.float64)
    return (Pm.T @ A_f @ Pm + sp.diags(1.0 - free_c)).tocsr()


class Hierarchy:
    """Level operators A_l, masks, prolongations and diagonals.  order0 is
    the element degree of the finest level: degree 3 coarsens first by 3
    (onto its vertex lattice), every other step halves the lattice; the
    multicolour Gauss-Seidel sweep of that level uses order0 + 1 colours
    per axis."""

    def __init__(self, A0, mask0, dims0, nlevels, order0=1):
        self.A = [A0.tocsr()]
        self.mask = [np.asarray(mask0, dtype=np.uint8)]
        self.dims = [tuple(dims0)]
        self.P = []
        self.gs_period = order0 + 1
        for l in range(1, nlevels):
            ratio = 3 if (l == 1 and order0 == 3) else 2
            dc = coarse_dims(self.dims[-1], ratio)
            mc = coarse_mask(self.mask[-1], self.dims[-1], ratio)
            Pm = masked_prolongation(dc, self.mask[-1], mc, ratio)
            self.P.append(Pm)
            self.A.append(galerkin(self.A[-1], Pm, mc))
            self.mask.append(mc)
            self.dims.append(dc)
        self.diag = [A.diagonal() for A in self.A]
        self.coarse_cho = sla.cho_factor(self.A[-1].toarray())

    @property
    def nlevels(self):
        return len(self.A)


def jacobi(A, wd, b, x):
    """One weighted-Jacobi sweep with per-DOF weights already divided by the
    diagonal."""
    return x + wd * (b - A @ x)


THETA = 1.9


def smoother_weights(H, omega, theta=THETA):
    """Per level, the per-DOF weight w_i / A_ii of the capped Jacobi sweep
    (0 on fixed DOFs, whose rows are identity)."""
    out = []
    for l in range(H.nlevels):
        A = H.A[l]
        d = H.diag[l]
        rs = np.asarray(abs(A).sum(axis=1)).ravel()
        w = np.minimum(omega, theta * d / rs)
        wd = w / d
        wd[np.asarray(H.mask[l]) != 0] = 0.0
        out.append(wd)
    return out


def node_colours(dims, period=3):
    """Colour (i mod m) + m (j mod m) + m^2 (k mod m), m = period, of every
    node of the lattice dims = (nx, ny, nz), x fastest."""
    nx, ny, nz = dims
    m = period
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i % m) + m * (j % m) + m * m * (k % m)).ravel()


def gs_order(dims, period=3):
    """The DOFs in forward sweep order: colour-major, then component, then
    node index."""
    col = node_colours(dims, period)
    out = []
    for c in range(period ** 3):
        nodes = np.nonzero(col == c)[0]
        for comp in range(3):
            out.append(3 * nodes + comp)
    return out


def gs_sweep(A, b, x, dims, backward=False, period=3):
    """One Gauss-Seidel sweep (relaxation 1) in multicolour order; every
    group of the order holds DOFs whose rows do not couple, so each group
    is updated at once from the latest values.  Fixed DOFs are identity
    rows with b = 0 and stay 0."""
    A = A.tocsr()
    d = A.diagonal()
    x = x.copy()
    groups = gs_order(dims, period)
    if backward:
        groups = groups[::-1]
    for idx in groups:
        x[idx] += (b[idx] - A[idx, :] @ x) / d[idx]
    return x


def vcycle(H, b, level=0, omega=0.6, pre=1, post=1, weights=None, smoother="jacobi"):
    """z = M b: Algorithm 1 recursively, from a zero initial guess, with the
    capped Jacobi weights (computed once per hierarchy when not given).
    smoother="gs": the multicolour Gauss-Seidel sweeps on the finest level
    (forward before, backward after the coarse correction)."""
    if weights is None:
        weights = getattr(H, "_weights", {}).get(omega)
        if weights is None:
            weights = smoother_weights(H, omega)
            H._weights = {omega: weights}
    if level == H.nlevels - 1:
        return sla.cho_solve(H.coarse_cho, b)
    A = H.A[level]
    wd = weights[level]
    gs = smoother == "gs" and level == 0
    x = np.zeros_like(b)
    m = getattr(H, "gs_period", 3)
    for _ in range(pre):
        x = gs_sweep(A, b, x, H.dims[0], period=m) if gs else jacobi(A, wd, b, x)
    r = b - A @ x
    e = vcycle(H, H.P[level].T @ r, level + 1, omega, pre, post, weights)
    x = x + H.P[level] @ e
    for _ in range(post):
        x = gs_sweep(A, b, x, H.dims[0], backward=True, period=m) if gs else jacobi(A, wd, b, x)
    return x


def mgcg(H, f, x0=None, rtol=1e-12, maxit=2000, omega=0.6, pre=1, post=1, smoother="jacobi"):
    """Preconditioned CG on A_0 x = f with M = vcycle; returns (x, iters,
    final true relative residual)."""
    A = H.A[0]
    x = np.zeros_like(f) if x0 is None else x0.copy()
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return np.zeros_like(f), 0, 0.0
    r = f - A @ x
    if np.linalg.norm(r) <= rtol * nf:
        return x, 0, np.linalg.norm(r) / nf
    z = vcycle(H, r, 0, omega, pre, post, smoother=smoother)
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * nf:
            r_true = f - A @ x
            if np.linalg.norm(r_true) <= rtol * nf:
                break
            r = r_true
        z = vcycle(H, r, 0, omega, pre, post, smoother=smoother)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.linalg.norm(f - A @ x) / nf
