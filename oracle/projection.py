"""Design-variable projection, density filter and their chain rule (plain definitions).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the product
path may import or call this module.

Lattices.  Displacement elements are unit cubes.  The density lattice has n
cells per element and axis, the design lattice d; both are C-order arrays of
shape (m*nelz, m*nely, m*nelx) with m = n or d, x fastest.  The centre of
density cell i is ((2 i_x + 1) / (2n), ...) and that of design cell j is
((2 j_x + 1) / (2d), ...).

* Filter weights, Sec. 2.2 eq. (4):
      omega_ij = exp(-dist(i, j)^2 / (2 (rmin/3)^2)) / (2 pi rmin/3)
  when dist(i, j) <= rmin, and 0 otherwise.
* Projection of the design variables onto the densities, Sec. 3.2 eq. (5):
      rho_i = sum_j (omega_ij / omega_i) x_j,   omega_i = sum_j omega_ij,
  the sums over the design cells of the domain.  With d = n this is the
  weighted-average density filter of Sec. 2.2 applied to x.
* Chain rule, Sec. 3.4: with W_ij = omega_ij / omega_i,
      df/dx_k = sum_i (df/drho_i) omega_ik / omega_i = (W^T g)_k,
  and the volume constraint's gradient is W^T v, v_i the density cells'
  volumes (1/n^3 here).

Reading (the test dist <= rmin decided exactly): along an axis the offset
between the centres of density cell i and design cell j is m / (2 n d) with
the integer m = (2 i + 1) d - (2 j + 1) n, so dist <= rmin is
m_x^2 + m_y^2 + m_z^2 <= (2 n d rmin)^2, the right side evaluated in FP64.

Pins (tests/test_oracle_projection.py): an all-pairs construction from
floating-point centre coordinates on tiny lattices; rows of W sum to one;
closed forms on two- and three-cell meshes (adjacent cells at exactly
dist = rmin are inside); the identity for d = n and rmin below the cell
spacing; W^T checked by central finite differences of the compliance
c(rho(x)) on a tiny mesh (the oracle's own solve).
"""

import math

import numpy as np
import scipy.sparse as sp


def lattice_shape(nel, m):
    """(z, y, x) shape of the lattice with m cells per element and axis."""
    return (m * nel[2], m * nel[1], m * nel[0])


def sigma(rmin):
    """The Gaussian's standard deviation rmin / 3 of eq. (4)."""
    return rmin / 3.0


def weight(dist2, rmin):
    """omega of eq. (4) for a squared centre distance inside the ball."""
    s = sigma(rmin)
    return math.exp(-dist2 / (2.0 * s * s)) / (2.0 * math.pi * s)


def _threshold(n, d, rmin):
    r = 2.0 * n * d * rmin
    return r * r


def _axis_pairs(ncell_rho, ncell_x, n, d, rmin):
    """Pairs (i, j, m) along one axis with |m| within the ball's radius."""
    i = np.arange(ncell_rho)[:, None]
    j = np.arange(ncell_x)[None, :]
    m = (2 * i + 1) * d - (2 * j + 1) * n
    ii, jj = np.nonzero(m.astype(np.float64) ** 2 <= _threshold(n, d, rmin))
    return ii, jj, m[ii, jj]


def weight_matrix(nel, n, d, rmin):
    """The unnormalised weights Omega (n_rho x n_x, sparse CSR): Omega_ij =
    omega_ij of eq. (4) over every (density, design) pair inside the ball."""
    Sr = lattice_shape(nel, n)
    Sx = lattice_shape(nel, d)
    pz = _axis_pairs(Sr[0], Sx[0], n, d, rmin)
    py = _axis_pairs(Sr[1], Sx[1], n, d, rmin)
    px = _axis_pairs(Sr[2], Sx[2], n, d, rmin)
    R2 = _threshold(n, d, rmin)
    scale = float(2 * n * d) ** 2
    rows, cols, vals = [], [], []
    for iz, jz, mz in zip(*pz):
        for iy, jy, my in zip(*py):
            ix, jx, mx = px
            M = (mx.astype(np.int64) ** 2 + int(my) ** 2 + int(mz) ** 2)
            keep = M.astype(np.float64) <= R2
            if not keep.any():
                continue
            r_idx = ix[keep] + Sr[2] * (iy + Sr[1] * iz)
            c_idx = jx[keep] + Sx[2] * (jy + Sx[1] * jz)
            w = np.array([weight(float(Mv) / scale, rmin) for Mv in M[keep]])
            rows.append(r_idx)
            cols.append(c_idx)
            vals.append(w)
    nr = Sr[0] * Sr[1] * Sr[2]
    nx = Sx[0] * Sx[1] * Sx[2]
    if not rows:
        return sp.csr_matrix((nr, nx))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nr, nx))


def projection_matrix(nel, n, d, rmin):
    """W = diag(1 / omega_i) Omega of eq. (5).  Raises if a density cell has no
    design cell inside its ball (omega_i = 0)."""
    Om = weight_matrix(nel, n, d, rmin)
    wi = np.asarray(Om.sum(axis=1)).ravel()
    if np.any(wi <= 0.0):
        raise ValueError("a density cell has no design cell within rmin")
    return sp.diags(1.0 / wi) @ Om


def project(x, nel, n, d, rmin):
    """rho = W x (eq. (5)), flat, in the density lattice's order."""
    return projection_matrix(nel, n, d, rmin) @ np.ravel(x)


def project_transpose(g, nel, n, d, rmin):
    """W^T g: the design-variable gradient of Sec. 3.4 from a density gradient."""
    return projection_matrix(nel, n, d, rmin).T @ np.ravel(g)


def volume_gradient(nel, n, d, rmin):
    """Gradient of sum_i v_i rho_i with respect to x (Sec. 3.4), v_i = 1/n^3."""
    nr = int(np.prod(lattice_shape(nel, n)))
    return project_transpose(np.full(nr, 1.0 / n ** 3), nel, n, d, rmin)


# ---- single entries, for sampled checks on full-size lattices ----

def _ball(i3, nel, n, d, rmin):
    """Design cells j inside the ball of density cell i3 = (ix, iy, iz) and
    their squared distances (exact integer test, FP64 distances)."""
    Sx = lattice_shape(nel, d)
    R2 = _threshold(n, d, rmin)
    axes = []
    for a, ia in enumerate(i3):
        ncx = Sx[2 - a]
        j = np.arange(ncx)
        m = (2 * ia + 1) * d - (2 * j + 1) * n
        ok = m.astype(np.float64) ** 2 <= R2
        axes.append((j[ok], m[ok].astype(np.int64)))
    (jx, mx), (jy, my), (jz, mz) = axes
    M = mx[None, None, :] ** 2 + my[None, :, None] ** 2 + mz[:, None, None] ** 2
    inside = M.astype(np.float64) <= R2
    kz, ky, kx = np.nonzero(inside)
    idx = jx[kx] + Sx[2] * (jy[ky] + Sx[1] * jz[kz])
    return idx, M[inside].astype(np.float64) / float(2 * n * d) ** 2


def omega_at(i3, nel, n, d, rmin):
    """omega_i of density cell i3."""
    _, d2 = _ball(i3, nel, n, d, rmin)
    return sum(weight(v, rmin) for v in d2)


def project_at(x, i3, nel, n, d, rmin):
    """rho_i of one density cell (eq. (5))."""
    x = np.ravel(x)
    idx, d2 = _ball(i3, nel, n, d, rmin)
    w = np.array([weight(v, rmin) for v in d2])
    return float(w @ x[idx]) / float(w.sum())


def project_transpose_at(g, k3, nel, n, d, rmin):
    """(W^T g)_k of one design cell k3 = (kx, ky, kz): sum over the density
    cells whose ball holds k of g_i omega_ik / omega_i."""
    g = np.ravel(g)
    Sr = lattice_shape(nel, n)
    R2 = _threshold(n, d, rmin)
    axes = []
    for a, ka in enumerate(k3):
        ncr = Sr[2 - a]
        i = np.arange(ncr)
        m = (2 * i + 1) * d - (2 * ka + 1) * n
        ok = m.astype(np.float64) ** 2 <= R2
        axes.append((i[ok], m[ok].astype(np.int64)))
    (ix, mx), (iy, my), (iz, mz) = axes
    total = 0.0
    scale = float(2 * n * d) ** 2
    for a, (cz, vz) in enumerate(zip(iz, mz)):
        for b, (cy, vy) in enumerate(zip(iy, my)):
            for cx, vx in zip(ix, mx):
                M = int(vx) ** 2 + int(vy) ** 2 + int(vz) ** 2
                if float(M) > R2:
                    continue
                i3 = (int(cx), int(cy), int(cz))
                flat = i3[0] + Sr[2] * (i3[1] + Sr[1] * i3[2])
                total += g[flat] * weight(M / scale, rmin) / omega_at(i3, nel, n, d, rmin)
    return total


__all__ = ["lattice_shape", "weight", "weight_matrix", "projection_matrix", "project",
           "project_transpose", "volume_gradient", "omega_at", "project_at",
           "project_transpose_at"]
