"""Structured-mesh bookkeeping, SIMP moduli and the sparse global stiffness.

* SIMP modulus of a density: E(rho) = Emin + rho^p (E0 - Emin) (Sec. 2,
  eq. (1); the modified form with a void floor Emin).
* Multiresolution element matrix: K^(e) = sum_i E(rho_{e_i}) K^(e_i) over the
  n^3 density sub-elements of displacement element e (Sec. 3.3, eq. (7)).
* Global K: superposition of the element matrices (Sec. 3.3), COO summation.
* Supports: the rows and columns of fixed DOFs are removed (Sec. 6.1); the
  HIP path equivalently keeps identity rows there, and ``level_operator``
  builds that form for comparisons.

Node numbering is lexicographic with x fastest (the paper is silent); the
density lattice is the C-order array (n*nelz, n*nely, n*nelx).
"""

import numpy as np
import scipy.sparse as sp


def node_dims(nel, order):
    return tuple(order * n + 1 for n in nel)


def element_dofs(nel, order):
    """Global DOF indices of every element, [nel_total, 3*n_e]; element
    e = ex + nelx*(ey + nely*ez)."""
    nelx, nely, nelz = nel
    nx, ny, _ = node_dims(nel, order)
    p1 = order + 1
    ez, ey, ex = np.meshgrid(np.arange(nelz), np.arange(nely), np.arange(nelx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    cols = []
    for az in range(p1):
        for ay in range(p1):
            for ax in range(p1):
                node = (order * ex + ax) + nx * ((order * ey + ay) + ny * (order * ez + az))
                for c in range(3):
                    cols.append(3 * node + c)
    return np.stack(cols, axis=1)


def density_index(nel, nsub):
    """Index into the flattened density lattice of every (element, sub-element)
    pair, [nel_total, n^3]; sub-element i = sx + n*(sy + n*sz)."""
    nelx, nely, nelz = nel
    n = nsub
    ez, ey, ex = np.meshgrid(np.arange(nelz), np.arange(nely), np.arange(nelx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    out = []
    for sz in range(n):
        for sy in range(n):
            for sx in range(n):
                ix, iy, iz = n * ex + sx, n * ey + sy, n * ez + sz
                out.append(ix + (n * nelx) * (iy + (n * nely) * iz))
    return np.stack(out, axis=1)


def simp_modulus(rho, E0=1.0, Emin=1e-9, penal=3.0):
    rho = np.asarray(rho, dtype=np.float64)
    return Emin + rho ** penal * (E0 - Emin)


def element_matrices(rho, nel, nsub, Ksub, E0=1.0, Emin=1e-9, penal=3.0):
    """K^(e) for every displacement element, [nel_total, nd, nd]."""
    E = simp_modulus(np.ravel(rho), E0, Emin, penal)
    Ee = E[density_index(nel, nsub)]                       # [nel, n^3]
    nd = Ksub.shape[1]
    return (Ee @ Ksub.reshape(Ksub.shape[0], nd * nd)).reshape(-1, nd, nd)


def assemble(Ke, nel, order):
    """Sparse global K (CSR) from element matrices."""
    edofs = element_dofs(nel, order)
    nd = edofs.shape[1]
    ndof = 3 * int(np.prod(node_dims(nel, order)))
    rows = np.repeat(edofs, nd, axis=1).ravel()
    cols = np.tile(edofs, (1, nd)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def stiffness(rho, nel, order, nsub, Ksub, E0=1.0, Emin=1e-9, penal=3.0):
    return assemble(element_matrices(rho, nel, nsub, Ksub, E0, Emin, penal), nel, order)


def apply(rho, nel, order, nsub, Ksub, u, E0=1.0, Emin=1e-9, penal=3.0, chunk=2048):
    """K u without forming K: the superposition of K^(e) u_e over the
    elements (the same sum that assembles K), element chunks at a time to
    bound memory.  u: [ndof] or [nrhs, ndof]."""
    u = np.atleast_2d(np.asarray(u, dtype=np.float64))
    edofs = element_dofs(nel, order)
    E = simp_modulus(np.ravel(rho), E0, Emin, penal)
    didx = density_index(nel, nsub)
    nd = Ksub.shape[1]
    Kflat = Ksub.reshape(Ksub.shape[0], nd * nd)
    y = np.zeros_like(u)
    for e0 in range(0, edofs.shape[0], chunk):
        ed = edofs[e0:e0 + chunk]
        Ke = (E[didx[e0:e0 + chunk]] @ Kflat).reshape(-1, nd, nd)
        for l in range(u.shape[0]):
            ye = np.einsum("eab,eb->ea", Ke, u[l][ed])
            y[l] += np.bincount(ed.ravel(), weights=ye.ravel(), minlength=u.shape[1])
    return y


def level_operator(K, mask):
    """Z K Z + (I - Z), Z = diag(free): the supported system written on all
    DOFs with identity rows at fixed DOFs."""
    free = (np.asarray(mask) == 0).astype(np.float64)
    Z = sp.diags(free)
    return (Z @ K @ Z + sp.diags(1.0 - free)).tocsr()
