"""Equilibrium solve, compliance and density gradient (plain definitions).

* u = K_ff^{-1} f_f with the supported DOFs removed (Sec. 2: K is positive
  definite once the supports are imposed, so the compliance is
  f^T K^{-1} f, problem (3)).  Dense Cholesky for small systems, sparse LU
  for medium ones, and for large ones the paper's own MGCG run to a tight
  tolerance (``multigrid.mgcg``).
* Compliance of load case l: c_l = f_l^T u_l (problem (2)); with several load
  cases the objective is their sum.
* Gradient with respect to a density (Sec. 3.4 with the design variables
  equal to the densities, i.e. without the chain factor omega_ik/omega_i):
  dc/drho_i = - p rho_i^{p-1} (E0 - Emin) * sum_l u_{l,e}^T K^(e_i) u_{l,e},
  where e is the displacement element containing density element i and
  u_{l,e} its nodal displacements.

Pins (tests/test_oracle_solve.py): compliance = f^T u = u^T K u; brute-force
dense solve of the full system with identity rows; patch test (a linear field
prescribed on the boundary is reproduced inside); the uniform-density
scaling c(r) = c(1) E0 / E(r); dc <= 0; the exact identity
sum_i rho_i dc_i = -p (c - Emin * sum_i u_e^T K^(e_i) u_e); central finite
differences on tiny meshes.
"""

import numpy as np
import scipy.sparse.linalg as spla
import scipy.linalg as sla

from .assemble import (element_dofs, density_index, simp_modulus, stiffness,
                       level_operator, node_dims)
from .multigrid import Hierarchy, mgcg


def solve_direct(K, mask, f):
    """u (all DOFs, zero at fixed ones) with K_ff u_f = f_f, per load case."""
    free = np.flatnonzero(np.asarray(mask) == 0)
    Kff = K[free][:, free]
    f = np.atleast_2d(f)
    u = np.zeros_like(f)
    if free.size <= 16000:
        cho = sla.cho_factor(Kff.toarray())
        for l in range(f.shape[0]):
            u[l, free] = sla.cho_solve(cho, f[l, free])
    else:
        lu = spla.splu(Kff.tocsc())
        for l in range(f.shape[0]):
            u[l, free] = lu.solve(f[l, free])
    return u


def solve_mgcg(K, mask, f, dims, nlevels, x0=None, rtol=1e-12, omega=0.6, maxit=2000, order=1):
    A0 = level_operator(K, mask)
    f = np.atleast_2d(f).copy()
    f[:, np.asarray(mask) != 0] = 0.0
    H = Hierarchy(A0, mask, dims, nlevels, order0=order)
    u = np.zeros_like(f)
    info = []
    for l in range(f.shape[0]):
        u[l], it, rr = mgcg(H, f[l], None if x0 is None else x0[l], rtol, maxit, omega)
        info.append((it, rr))
    return u, info


def compliance(f, u):
    """Per-load-case compliance f_l^T u_l."""
    return np.einsum("ld,ld->l", np.atleast_2d(f), np.atleast_2d(u))


def sub_energies(u, nel, order, Ksub):
    """u_e^T K^(e_i) u_e summed over load cases, [nel_total, n^3]."""
    edofs = element_dofs(nel, order)
    out = 0.0
    for ul in np.atleast_2d(u):
        ue = ul[edofs]                                      # [nel, nd]
        out = out + np.einsum("ea,sab,eb->es", ue, Ksub, ue, optimize=True)
    return out


def sensitivity(rho, u, nel, order, nsub, Ksub, E0=1.0, Emin=1e-9, penal=3.0):
    """dc/drho in the density lattice's flat order."""
    rho = np.ravel(rho)
    w = sub_energies(u, nel, order, Ksub)                  # [nel, n^3]
    dc = np.zeros_like(rho)
    idx = density_index(nel, nsub)
    dc[idx.ravel()] = -penal * rho[idx.ravel()] ** (penal - 1) * (E0 - Emin) * w.ravel()
    return dc


def solve_problem(rho, mask, f, nel, order, nsub, Ksub, E0=1.0, Emin=1e-9, penal=3.0,
                  method="direct", nlevels=3, rtol=1e-12):
    """Convenience: K, u, per-case compliance and dc."""
    K = stiffness(rho, nel, order, nsub, Ksub, E0, Emin, penal)
    if method == "direct":
        u = solve_direct(K, mask, f)
    else:
        u, _ = solve_mgcg(K, mask, f, node_dims(nel, order), nlevels, rtol=rtol, order=order)
    c = compliance(f, u)
    dc = sensitivity(rho, u, nel, order, nsub, Ksub, E0, Emin, penal)
    return K, u, c, dc


__all__ = ["solve_direct", "solve_mgcg", "compliance", "sub_energies", "sensitivity",
           "solve_problem", "simp_modulus"]
