"""Pins of the oracle's assembly, solve, compliance and gradient."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble, fem, solve

MAT = dict(E0=1.0, Emin=1e-9, penal=3.0)


def _setup(nel, order, nsub, kind="cantilever", nrhs=1, seed=0):
    mask, f = W.make_problem(kind, *nel, order, nrhs)
    n = nsub
    rho = W.uniform_field((nel[2] * n, nel[1] * n, nel[0] * n), seed, 0.1, 1.0)
    Ks = fem.sub_element_matrices(order, nsub)
    return mask, f, rho, Ks


def test_brute_force_dense_solve():
    """The supported system solved by numpy on all DOFs with identity rows
    equals the oracle's eliminated solve."""
    for nel, order, nsub in [((1, 1, 1), 1, 1), ((2, 1, 1), 1, 1), ((3, 2, 2), 1, 2),
                             ((1, 1, 1), 2, 1), ((2, 1, 1), 2, 2)]:
        mask, f, rho, Ks = _setup(nel, order, nsub, nrhs=2)
        K = assemble.stiffness(rho, nel, order, nsub, Ks, **MAT)
        u = solve.solve_direct(K, mask, f)
        A = assemble.level_operator(K, mask).toarray()
        ub = np.linalg.solve(A, f.T).T
        assert np.abs(u - ub).max() <= 1e-10 * np.abs(ub).max()


def test_compliance_identity():
    """c = f^T u = u^T K u (Sec. 3.4)."""
    mask, f, rho, Ks = _setup((4, 2, 2), 1, 2, nrhs=3)
    K, u, c, dc = solve.solve_problem(rho, mask, f, (4, 2, 2), 1, 2, Ks, **MAT)
    cu = np.einsum("ld,ld->l", u, (K @ u.T).T)
    assert np.allclose(c, cu, rtol=1e-12)
    assert np.all(c > 0)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_patch_test(order):
    """Uniform material, a linear field prescribed on the boundary and no
    loads: the solution reproduces the linear field at interior nodes."""
    nel = (3, 3, 2)
    dims = assemble.node_dims(nel, order)
    Ks = fem.sub_element_matrices(order, 1)
    K = assemble.stiffness(np.ones((2, 3, 3)), nel, order, 1, Ks, **MAT)
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], 1) / order
    grad = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [0.2, 0.1, -0.15]])
    u_lin = (X @ grad.T + np.array([0.1, -0.2, 0.3])).ravel()
    bnd = ((i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1) | (k == 0) | (k == nz - 1)).ravel()
    fixed = np.repeat(bnd, 3)
    free = ~fixed
    Kd = K.toarray()
    u = u_lin.copy()
    u[free] = np.linalg.solve(Kd[np.ix_(free, free)], -Kd[np.ix_(free, fixed)] @ u_lin[fixed])
    assert free.sum() > 0
    assert np.abs(u - u_lin).max() < 1e-12
    # a linear field leaves zero force on interior nodes
    assert np.abs((Kd @ u_lin)[free]).max() < 1e-12


def test_uniform_density_scaling():
    """K(rho = r) = E(r)/E0 * K(rho = 1), so c(r) = c(1) * E0 / E(r)."""
    nel = (4, 2, 2)
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    Ks = fem.sub_element_matrices(1, 1)
    c1 = solve.solve_problem(np.ones((2, 2, 4)), mask, f, nel, 1, 1, Ks, **MAT)[2]
    r = 0.37
    cr = solve.solve_problem(np.full((2, 2, 4), r), mask, f, nel, 1, 1, Ks, **MAT)[2]
    Er = MAT["Emin"] + r ** 3 * (MAT["E0"] - MAT["Emin"])
    assert abs(cr[0] - c1[0] / Er) < 1e-10 * cr[0]


def test_multiresolution_reduces_to_single_resolution():
    """With all n^3 sub-densities of an element equal to its density, eq. (7)
    gives the single-resolution element of eq. (1)."""
    nel = (3, 2, 2)
    rho1 = W.uniform_field((2, 2, 3), 3, 0.1, 1.0)
    rho2 = np.repeat(np.repeat(np.repeat(rho1, 2, 0), 2, 1), 2, 2)
    K1 = assemble.stiffness(rho1, nel, 1, 1, fem.sub_element_matrices(1, 1), **MAT)
    K2 = assemble.stiffness(rho2, nel, 1, 2, fem.sub_element_matrices(1, 2), **MAT)
    assert abs(K1 - K2).max() < 1e-14


def test_timoshenko_beam():
    """Slender clamped beam under a unit tip load: the compliance (= tip
    deflection) of Q2 elements within 2% of Timoshenko beam theory, Q1 within
    6% on a finer mesh (Q1 elements are stiffer in bending)."""
    for order, (L, h, b), tol in [(2, (20, 2, 2), 0.02), (1, (40, 4, 4), 0.06)]:
        EI = b * h ** 3 / 12.0
        GA = 5.0 / 6.0 * b * h / (2 * 1.3)
        tim = L ** 3 / (3 * EI) + L / GA
        mask, f = W.make_problem("cantilever", L, h, b, order, 1)
        Ks = fem.sub_element_matrices(order, 1)
        c = solve.solve_problem(np.ones((b, h, L)), mask, f, (L, h, b), order, 1, Ks,
                                E0=1.0, Emin=0.0, penal=3.0)[2][0]
        assert abs(c / tim - 1) < tol


def test_sensitivity_sign_and_identity():
    """dc <= 0, and from eq. (7): sum_i rho_i dc_i = -p (c - Emin sum_i
    u_e^T K^(e_i) u_e) (one load case)."""
    nel, order, nsub = (4, 2, 2), 1, 2
    mask, f, rho, Ks = _setup(nel, order, nsub, nrhs=2)
    K, u, c, dc = solve.solve_problem(rho, mask, f, nel, order, nsub, Ks, **MAT)
    assert np.all(dc <= 0)
    for l in range(2):
        ul = u[l:l + 1]
        dcl = solve.sensitivity(rho, ul, nel, order, nsub, Ks, **MAT)
        w = solve.sub_energies(ul, nel, order, Ks).sum()
        lhs = np.sum(rho.ravel() * dcl)
        rhs = -MAT["penal"] * (c[l] - MAT["Emin"] * w)
        assert abs(lhs - rhs) < 1e-11 * abs(rhs)


@pytest.mark.parametrize("nel,order,nsub", [((2, 1, 1), 1, 2), ((1, 1, 1), 2, 2),
                                            ((3, 1, 2), 1, 1), ((1, 1, 1), 3, 2)])
def test_sensitivity_central_differences(nel, order, nsub):
    """Entrywise central differences (h = 1e-6) of c = sum_l f_l^T u_l."""
    mask, f, rho, Ks = _setup(nel, order, nsub, nrhs=2, seed=5)
    _, _, c, dc = solve.solve_problem(rho, mask, f, nel, order, nsub, Ks, **MAT)
    h = 1e-6
    flat = rho.ravel()
    for i in range(flat.size):
        rp, rm = flat.copy(), flat.copy()
        rp[i] += h
        rm[i] -= h
        cp = solve.solve_problem(rp.reshape(rho.shape), mask, f, nel, order, nsub, Ks, **MAT)[2].sum()
        cm = solve.solve_problem(rm.reshape(rho.shape), mask, f, nel, order, nsub, Ks, **MAT)[2].sum()
        fd = (cp - cm) / (2 * h)
        assert abs(fd - dc[i]) <= 1e-6 * abs(c.sum()) + 1e-6 * abs(dc[i])


def test_rigid_modes_of_unsupported_assembly():
    """The assembled K without supports has the six rigid-body modes in its
    null space."""
    nel = (3, 2, 2)
    Ks = fem.sub_element_matrices(1, 2)
    rho = W.uniform_field((4, 4, 6), 9, 0.1, 1.0)
    K = assemble.stiffness(rho, nel, 1, 2, Ks, **MAT)
    nx, ny, nz = assemble.node_dims(nel, 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], 1).astype(float)
    R = fem.rigid_body_modes(X)
    assert np.abs(K @ R.T).max() < 1e-12
    # and the supported operator is positive definite
    A = assemble.level_operator(K, W.make_problem("cantilever", *nel, 1, 1)[0])
    assert spla.eigsh(A, k=1, which="SA", return_eigenvectors=False)[0] > 0


@pytest.mark.parametrize("order,nsub", [(1, 1), (1, 2), (2, 2), (3, 1)])
def test_elementwise_apply(order, nsub):
    """K u without forming K: rigid-body modes give zero force, a linear
    field gives zero force at interior nodes (patch test), the map is
    symmetric, and it equals the assembled K (small chunks exercise the
    chunk loop)."""
    nel = (3, 2, 2)
    mask, f, rho, Ks = _setup(nel, order, nsub, seed=4)
    dims = assemble.node_dims(nel, order)
    nx, ny, nz = dims
    z, y, x = np.meshgrid(*(np.arange(d, dtype=float) / (d - 1) for d in (nz, ny, nx)),
                          indexing="ij")
    x, y, z = x.ravel() * nel[0], y.ravel() * nel[1], z.ravel() * nel[2]
    modes = []
    for c in range(3):
        m = np.zeros((x.size, 3))
        m[:, c] = 1.0
        modes.append(m.ravel())
    for a, b, p, q in [(0, 1, x, y), (1, 2, y, z), (2, 0, z, x)]:
        m = np.zeros((x.size, 3))
        m[:, a], m[:, b] = -q, p
        modes.append(m.ravel())
    for m in modes:
        r = assemble.apply(rho, nel, order, nsub, Ks, m, chunk=5, **MAT)
        assert np.abs(r).max() <= 1e-12 * np.abs(m).max()
    # patch test: a linear field (uniform strain) balances at interior nodes
    lin = np.stack([0.3 * x - 0.2 * y, 0.1 * y + 0.4 * z, -0.25 * z + 0.05 * x], axis=1).ravel()
    r = assemble.apply(np.ones_like(rho), nel, order, nsub, Ks, lin, **MAT).reshape(-1, 3)
    interior = ((x > 0) & (x < nel[0]) & (y > 0) & (y < nel[1]) & (z > 0) & (z < nel[2]))
    assert interior.any()
    assert np.abs(r[interior]).max() <= 1e-12 * np.abs(r).max()
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, lin.size))
    Ku = assemble.apply(rho, nel, order, nsub, Ks, u, chunk=7, **MAT)[0]
    Kv = assemble.apply(rho, nel, order, nsub, Ks, v, **MAT)[0]
    assert abs(v @ Ku - u @ Kv) <= 1e-12 * abs(v @ Ku)
    K = assemble.stiffness(rho, nel, order, nsub, Ks, **MAT)
    assert np.abs(Ku - K @ u).max() <= 1e-12 * np.abs(Ku).max()
