"""Pins of the oracle's multigrid components."""

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assemble, fem, multigrid, solve

MAT = dict(E0=1.0, Emin=1e-9, penal=3.0)


def test_prolongation_reproduces_multilinear_fields():
    """Trilinear interpolation is exact for fields that are linear in each
    coordinate separately."""
    dc = (4, 3, 3)
    P = multigrid.prolongation(dc)
    df = tuple(2 * (d - 1) + 1 for d in dc)

    def field(dims, scale):
        nx, ny, nz = dims
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        x, y, z = i.ravel() * scale, j.ravel() * scale, k.ravel() * scale
        return np.stack([(1 + 0.3 * x) * (2 - 0.1 * y) * (0.5 + z),
                         x * y * z - 2 * x + 3,
                         (x - 1) * (z + 0.25)], 1).ravel()

    assert np.abs(P @ field(dc, 1.0) - field(df, 0.5)).max() < 1e-12
    # each fine node's weights sum to one (partition of unity)
    assert np.allclose(np.asarray(P.sum(1)).ravel(), 1.0)


def test_ratio_three_prolongation_reproduces_multilinear_fields():
    """The cubic lattice's first coarsening (onto its vertex lattice, every
    third node): the same exactness for multilinear fields, with the fine
    node q/3 of the way between two coarse nodes weighted 1 - q/3, q/3."""
    dc = (3, 2, 4)
    P = multigrid.prolongation(dc, 3)
    df = tuple(3 * (d - 1) + 1 for d in dc)
    assert P.shape == (3 * np.prod(df), 3 * np.prod(dc))

    def field(dims, scale):
        nx, ny, nz = dims
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        x, y, z = i.ravel() * scale, j.ravel() * scale, k.ravel() * scale
        return np.stack([(1 + 0.3 * x) * (2 - 0.1 * y) * (0.5 + z),
                         x * y * z - 2 * x + 3,
                         (x - 1) * (z + 0.25)], 1).ravel()

    assert np.abs(P @ field(dc, 1.0) - field(df, 1.0 / 3.0)).max() < 1e-12
    assert np.allclose(np.asarray(P.sum(1)).ravel(), 1.0)
    P1 = multigrid.prolong_1d(2, 3).toarray()
    assert np.allclose(P1, [[1, 0], [2 / 3, 1 / 3], [1 / 3, 2 / 3], [0, 1]])


def test_galerkin_of_constant_modulus_is_rediscretisation():
    """For uniform E and no supports, P^T K_h P equals the operator assembled
    from elements of twice the size (which in 3-D is 2 * K0 per element)."""
    nel = (4, 2, 2)
    Ks = fem.sub_element_matrices(1, 1)
    Kh = assemble.stiffness(np.ones((2, 2, 4)), nel, 1, 1, Ks, **MAT)
    P = multigrid.prolongation(assemble.node_dims((2, 1, 1), 1))
    KH = assemble.assemble(np.repeat(2.0 * Ks, 2, axis=0), (2, 1, 1), 1)
    assert abs(P.T @ Kh @ P - KH).max() < 1e-13


def test_galerkin_masked_definition():
    """A_c = P~^T A_f P~ + (I - Z_c): symmetric, identity on coarse fixed DOFs,
    and the coarse system restricted to free DOFs is positive definite."""
    nel = (4, 4, 2)
    mask, f = W.make_problem("mbb", *nel, 1, 1)
    rho = W.uniform_field((2, 4, 4), 2, 0.1, 1.0)
    K = assemble.stiffness(rho, nel, 1, 1, fem.sub_element_matrices(1, 1), **MAT)
    A0 = assemble.level_operator(K, mask)
    H = multigrid.Hierarchy(A0, mask, assemble.node_dims(nel, 1), 2)
    Ac = H.A[1].toarray()
    assert np.abs(Ac - Ac.T).max() < 1e-15
    mc = H.mask[1].astype(bool)
    assert np.allclose(Ac[np.ix_(mc, mc)], np.eye(mc.sum()))
    assert np.abs(Ac[np.ix_(mc, ~mc)]).max() == 0
    assert np.linalg.eigvalsh(Ac[np.ix_(~mc, ~mc)]).min() > 0


def _vcycle_matrix(H, mask, omega):
    n = H.A[0].shape[0]
    free = np.flatnonzero(mask == 0)
    Mm = np.zeros((n, n))
    for i in free:
        e = np.zeros(n)
        e[i] = 1.0
        Mm[:, i] = multigrid.vcycle(H, e, omega=omega)
    return Mm[np.ix_(free, free)]


def test_capped_smoother_converges_where_plain_omega_diverges():
    """On an i.i.d. rough field lambda_max(D^-1 A) > 2/0.6: the plain sweep
    with omega = 0.6 has spectral radius > 1, the capped one < 1, and the
    V-cycle built on it is symmetric positive definite."""
    nel = (4, 2, 2)
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    rho = W.uniform_field((2, 2, 4), 4, 0.001, 1.0)
    K = assemble.stiffness(rho, nel, 1, 1, fem.sub_element_matrices(1, 1), **MAT)
    H = multigrid.Hierarchy(assemble.level_operator(K, mask), mask,
                            assemble.node_dims(nel, 1), 2)
    free = np.flatnonzero(mask == 0)
    A = H.A[0].toarray()[np.ix_(free, free)]
    d = np.diag(A)
    plain = np.eye(len(free)) - 0.6 * A / d[:, None]
    assert np.abs(np.linalg.eigvals(plain)).max() > 1.0
    wd = multigrid.smoother_weights(H, 0.6)[0][free]
    capped = np.eye(len(free)) - wd[:, None] * A
    assert np.abs(np.linalg.eigvals(capped)).max() < 1.0
    # weights never exceed omega and keep it where the bound allows
    w = wd * d
    assert np.all(w <= 0.6 + 1e-15) and np.all(w > 0)
    Mf = _vcycle_matrix(H, mask, 0.6)
    assert np.abs(Mf - Mf.T).max() < 1e-10 * np.abs(Mf).max()
    assert np.linalg.eigvalsh(0.5 * (Mf + Mf.T)).min() > 0


def test_capped_weights_keep_omega_on_smooth_operators():
    """Where sum_j |A_ij| <= theta A_ii / omega the weight is omega itself."""
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 4.0]]))

    class _H:
        pass
    H = _H()
    H.A, H.diag, H.mask, H.nlevels = [A], [A.diagonal()], [np.zeros(3, np.uint8)], 1
    wd = multigrid.smoother_weights(H, 0.6)[0]
    assert np.allclose(wd * 4.0, 0.6)


@pytest.mark.parametrize("kind,order,nel,nlev", [("cantilever", 1, (8, 4, 4), 3),
                                                 ("mbb", 1, (8, 4, 4), 3),
                                                 ("cantilever", 2, (4, 2, 2), 3)])
def test_mgcg_matches_direct(kind, order, nel, nlev):
    mask, f = W.make_problem(kind, *nel, order, 2)
    rho = W.gaussian_random_field((nel[2] * 2, nel[1] * 2, nel[0] * 2), 7, corr=3.0)
    Ks = fem.sub_element_matrices(order, 2)
    K = assemble.stiffness(rho, nel, order, 2, Ks, **MAT)
    ud = solve.solve_direct(K, mask, f)
    um, info = solve.solve_mgcg(K, mask, f, assemble.node_dims(nel, order), nlev, rtol=1e-10,
                                omega=0.5)
    for l in range(2):
        assert info[l][1] <= 1e-10
        assert np.linalg.norm(um[l] - ud[l]) <= 1e-7 * np.linalg.norm(ud[l])


def _rough_hierarchy(nel, nlev, seed=4):
    mask, _ = W.make_problem("cantilever", *nel, 1, 1)
    rho = W.uniform_field((nel[2], nel[1], nel[0]), seed, 0.001, 1.0)
    K = assemble.stiffness(rho, nel, 1, 1, fem.sub_element_matrices(1, 1), **MAT)
    H = multigrid.Hierarchy(assemble.level_operator(K, mask), mask,
                            assemble.node_dims(nel, 1), nlev)
    return H, mask


def _cubic_hierarchy(nel, nlev, family="lagrange", seed=6, nsub=1):
    mask, f = W.make_problem("cantilever", *nel, 3, 1)
    if family == "serendipity":
        mask = np.maximum(mask, fem.serendipity_dof_mask(nel, 3))
    rho = W.uniform_field((nsub * nel[2], nsub * nel[1], nsub * nel[0]), seed, 0.001, 1.0)
    K = assemble.stiffness(rho, nel, 3, nsub, fem.sub_element_matrices(3, nsub, family=family),
                           **MAT)
    H = multigrid.Hierarchy(assemble.level_operator(K, mask), mask, assemble.node_dims(nel, 3),
                            nlev, order0=3)
    b = f[0].copy()
    b[mask.astype(bool)] = 0.0
    return H, mask, b


def _vcycle_full(H, **kw):
    n = H.A[0].shape[0]
    return np.stack([multigrid.vcycle(H, e, **kw) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("nel,nlev", [((4, 2, 2), 2), ((8, 4, 4), 3)])
def test_coarse_correction_is_an_a_orthogonal_projector(nel, nlev):
    """Algorithm 1 without smoothing (pre = post = 0) is the coarse-grid
    correction alone: M = Q A_c^-1 Q^T with Q the product of the masked
    prolongations and A_c = Q^T A Q on the coarse free DOFs (Galerkin,
    Sec. 2.3).  Then M A is the A-orthogonal projector onto range(Q): it is
    idempotent, A M A is symmetric, and M A reproduces every coarse field.
    A restriction or prolongation off by a factor (full weighting's 1/8, say)
    scales M A and breaks idempotency."""
    H, mask = _rough_hierarchy(nel, nlev)
    A = H.A[0].toarray()
    Mm = _vcycle_full(H, pre=0, post=0)
    MA = Mm @ A
    scale = np.abs(MA).max()
    assert np.abs(MA @ MA - MA).max() < 1e-9 * scale
    AMA = A @ MA
    assert np.abs(AMA - AMA.T).max() < 1e-9 * np.abs(AMA).max()
    Q = H.P[0].toarray()
    for P in H.P[1:]:
        Q = Q @ P.toarray()
    free_c = np.flatnonzero(H.mask[-1] == 0)
    Qf = Q[:, free_c]
    assert np.abs(MA @ Qf - Qf).max() < 1e-9 * max(1.0, np.abs(Qf).max())
    # the projector's rank is the number of free coarsest DOFs
    assert np.linalg.matrix_rank(MA, tol=1e-8 * scale) == len(free_c)


@pytest.mark.parametrize("family", ["lagrange", "serendipity"])
def test_cubic_coarse_correction_is_an_a_orthogonal_projector(family):
    """The same projector identity for a cubic finest level, whose first
    coarsening takes every third lattice node: a transfer with the wrong
    weights or scale would break it."""
    H, mask, _ = _cubic_hierarchy((2, 2, 2), 2, family)
    assert H.dims[1] == (3, 3, 3)
    A = H.A[0].toarray()
    Mm = _vcycle_full(H, pre=0, post=0)
    MA = Mm @ A
    scale = np.abs(MA).max()
    assert np.abs(MA @ MA - MA).max() < 1e-9 * scale
    AMA = A @ MA
    assert np.abs(AMA - AMA.T).max() < 1e-9 * np.abs(AMA).max()
    Qf = H.P[0].toarray()[:, np.flatnonzero(H.mask[1] == 0)]
    assert np.abs(MA @ Qf - Qf).max() < 1e-9 * max(1.0, np.abs(Qf).max())
    assert np.linalg.matrix_rank(MA, tol=1e-8 * scale) == Qf.shape[1]


def test_two_grid_error_propagation_composes_the_steps():
    """Algorithm 1 on two levels, one pre- and one post-sweep from x = 0:
    the error propagator I - M A is the product (I - S A)(I - C A)(I - S A)
    of the weighted-Jacobi sweep S = W D^-1 and the exact coarse correction
    C (itself the projector above), in that order."""
    H, mask = _rough_hierarchy((4, 2, 2), 2)
    A = H.A[0].toarray()
    n = A.shape[0]
    wd = multigrid.smoother_weights(H, 0.6)[0]
    S = np.eye(n) - wd[:, None] * A
    C = _vcycle_full(H, pre=0, post=0)
    Mm = _vcycle_full(H, pre=1, post=1, omega=0.6)
    lhs = np.eye(n) - Mm @ A
    rhs = S @ (np.eye(n) - C @ A) @ S
    assert np.abs(lhs - rhs).max() < 1e-9


def _q2_hierarchy(nel, nsub, nlev, seed=5, family="lagrange"):
    mask, f = W.make_problem("cantilever", *nel, 2, 1)
    if family == "serendipity":
        mask = np.maximum(mask, fem.serendipity_dof_mask(nel))
    rho = W.gaussian_random_field((nsub * nel[2], nsub * nel[1], nsub * nel[0]), seed, corr=3.0)
    K = assemble.stiffness(rho, nel, 2, nsub, fem.sub_element_matrices(2, nsub, family=family), **MAT)
    A0 = assemble.level_operator(K, mask)
    H = multigrid.Hierarchy(A0, mask, assemble.node_dims(nel, 2), nlev, order0=2)
    b = f[0].copy()
    b[mask.astype(bool)] = 0.0
    return H, mask, b


@pytest.mark.parametrize("order,nel,nsub", [(2, (2, 2, 2), 1), (2, (4, 2, 2), 2),
                                            (2, (3, 2, 3), 1), (3, (2, 2, 1), 1),
                                            (3, (1, 2, 2), 2)])
def test_gs_sweep_is_the_triangular_solve(order, nel, nsub):
    """A Gauss-Seidel sweep with relaxation 1 in a given order is
    x + (D + L)^-1 (b - A x), L the strictly lower triangle of A with rows
    and columns in that order (the backward sweep: the upper triangle).  The
    oracle updates a whole colour-component group at once, which equals the
    sequential sweep only if the group's rows do not couple: an order whose
    colours repeat every two nodes would fail."""
    from scipy.sparse.linalg import spsolve_triangular
    if order == 2:
        H, mask, _ = _q2_hierarchy(nel, nsub, 1)
    else:
        H, mask, _ = _cubic_hierarchy(nel, 1, nsub=nsub)
    m = order + 1
    assert H.gs_period == m
    A = H.A[0].tocsr()
    n = A.shape[0]
    rng = np.random.default_rng(11)
    b = rng.standard_normal(n)
    x = rng.standard_normal(n)
    b[mask.astype(bool)] = 0.0
    x[mask.astype(bool)] = 0.0
    perm = np.concatenate(multigrid.gs_order(H.dims[0], m))
    assert np.array_equal(np.sort(perm), np.arange(n))
    Ap = A[perm][:, perm].tocsr()
    r = (b - A @ x)[perm]
    lower = sp.tril(Ap, format="csr")
    upper = sp.triu(Ap, format="csr")
    want_f = x.copy()
    want_f[perm] += spsolve_triangular(lower, r, lower=True)
    want_b = x.copy()
    want_b[perm] += spsolve_triangular(upper, r, lower=False)
    got_f = multigrid.gs_sweep(A, b, x, H.dims[0], period=m)
    got_b = multigrid.gs_sweep(A, b, x, H.dims[0], backward=True, period=m)
    scale = np.abs(want_f).max()
    assert np.abs(got_f - want_f).max() <= 1e-11 * scale
    assert np.abs(got_b - want_b).max() <= 1e-11 * np.abs(want_b).max()
    # the colour classes of the lattice do not couple, while a period of
    # one less than order + 1 would put coupled nodes in one class
    col = multigrid.node_colours(H.dims[0], m)
    for c in range(m ** 3):
        nodes = np.flatnonzero(col == c)
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        blk = A[dofs][:, dofs].tocoo()
        assert np.all(blk.row // 3 == blk.col // 3)
    col = multigrid.node_colours(H.dims[0], m - 1)
    coupled = False
    for c in range((m - 1) ** 3):
        nodes = np.flatnonzero(col == c)
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        blk = A[dofs][:, dofs].tocoo()
        coupled |= bool(np.any((blk.row // 3 != blk.col // 3) & (blk.data != 0)))
    assert coupled


@pytest.mark.parametrize("family", ["lagrange", "serendipity"])
def test_gs_vcycle_is_spd_and_beats_jacobi(family):
    """The V-cycle with the forward sweep before and the backward sweep after
    the coarse correction is symmetric positive definite (the backward sweep
    is the forward one's adjoint), and MG-CG with it reaches the direct
    solve, on a rough field, in fewer iterations than with the capped Jacobi
    sweep (Sec. 7.5)."""
    H, mask, b = _q2_hierarchy((4, 2, 2), 2, 2, family=family)
    Mm = _vcycle_full(H, smoother="gs")
    assert np.abs(Mm - Mm.T).max() <= 1e-10 * np.abs(Mm).max()
    free = np.flatnonzero(mask == 0)
    ev = np.linalg.eigvalsh(0.5 * (Mm + Mm.T)[np.ix_(free, free)])
    assert ev.min() > 0.0
    xd = np.zeros_like(b)
    xd[free] = np.linalg.solve(H.A[0].toarray()[np.ix_(free, free)], b[free])
    xg, itg, res = multigrid.mgcg(H, b, rtol=1e-10, smoother="gs")
    _, itj, _ = multigrid.mgcg(H, b, rtol=1e-10)
    assert res <= 1e-10
    assert np.linalg.norm(xg - xd) <= 1e-8 * np.linalg.norm(xd)
    assert itg < itj


@pytest.mark.parametrize("family", ["lagrange", "serendipity"])
def test_cubic_gs_vcycle_is_spd_and_mgcg_reaches_the_direct_solve(family):
    """The cubic hierarchy (first coarsening by 3, then halving) with the
    4-colour-per-axis Gauss-Seidel sweep: the V-cycle is symmetric positive
    definite, and MG-CG with either smoother reaches the direct solve."""
    H, mask, b = _cubic_hierarchy((2, 1, 1), 2, family)
    Mm = _vcycle_full(H, smoother="gs")
    assert np.abs(Mm - Mm.T).max() <= 1e-10 * np.abs(Mm).max()
    free = np.flatnonzero(mask == 0)
    assert np.linalg.eigvalsh(0.5 * (Mm + Mm.T)[np.ix_(free, free)]).min() > 0.0
    xd = np.zeros_like(b)
    xd[free] = np.linalg.solve(H.A[0].toarray()[np.ix_(free, free)], b[free])
    for sm in ("gs", "jacobi"):
        x, it, res = multigrid.mgcg(H, b, rtol=1e-11, smoother=sm, maxit=4000)
        assert res <= 1e-11
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_cubic_mgcg_three_levels_matches_direct():
    """Three levels (cubic -> vertex lattice -> halved) on an MBB-type
    support with two load cases, through the oracle's solve entry."""
    nel = (4, 2, 2)
    mask, f = W.make_problem("mbb", *nel, 3, 2)
    rho = W.gaussian_random_field((2 * nel[2], 2 * nel[1], 2 * nel[0]), 8, corr=3.0)
    Ks = fem.sub_element_matrices(3, 2)
    K = assemble.stiffness(rho, nel, 3, 2, Ks, **MAT)
    ud = solve.solve_direct(K, mask, f)
    um, info = solve.solve_mgcg(K, mask, f, assemble.node_dims(nel, 3), 3, rtol=1e-10,
                                omega=0.5, order=3)
    for l in range(2):
        assert info[l][1] <= 1e-10
        assert np.linalg.norm(um[l] - ud[l]) <= 1e-7 * np.linalg.norm(ud[l])
