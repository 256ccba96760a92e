"""Kernel parity: every multigrid component of the HIP path against the
oracle's explicit sparse operators, on small meshes spanning several thread
blocks and ragged tails."""

import numpy as np
import pytest

from helpers import MAT, Case, need_gpu, rel

pytestmark = pytest.mark.gpu

CASES = [
    # kind, nel, order, nsub, nlevels, nrhs
    ("cantilever", (8, 4, 4), 1, 1, 3, 1),
    ("mbb", (12, 8, 4), 1, 1, 3, 2),
    ("torsion", (8, 4, 6), 1, 2, 2, 1),
    ("cantilever", (6, 2, 4), 2, 2, 3, 2),
    ("mbb", (4, 4, 2), 2, 1, 2, 1),
    # a stencil level above the fused-prolongation size and a coarsest level
    # above the fused-restriction size: the separate transfer kernels
    ("torsion", (64, 32, 32), 1, 2, 3, 1),
]


def _id(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-q{c[2]}-n{c[3]}-L{c[4]}-r{c[5]}"


@pytest.fixture(scope="module", params=CASES, ids=_id)
def case(request):
    need_gpu()
    kind, nel, order, nsub, nlev, nrhs = request.param
    c = Case(kind, nel, order, nsub, nlev, nrhs, seed=11)
    p = c.problem()
    p.set_densities(c.rho)
    yield c, p
    p.close()


def _rand(n, nrhs, seed):
    return np.random.default_rng(seed).standard_normal((nrhs, n))


def test_fine_apply_fp64(case):
    c, p = case
    x = _rand(p.ndof, c.nrhs, 1)
    y = p.apply(0, x)
    ref = (c.H.A[0] @ x.T).T
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


def test_coarse_applies_and_diagonals(case):
    c, p = case
    for l in range(c.nlevels):
        (_, n) = p.level_dims(l)
        x = _rand(n, c.nrhs, 2 + l)
        y = p.apply(l, x)
        ref = (c.H.A[l] @ x.T).T
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max(), l
        d = p.diag(l)
        assert np.abs(d - c.H.diag[l]).max() <= 1e-13 * np.abs(c.H.diag[l]).max(), l


def test_transfers(case):
    c, p = case
    for l in range(c.nlevels - 1):
        nf = p.level_dims(l)[1]
        nc = p.level_dims(l + 1)[1]
        xf = _rand(nf, c.nrhs, 5 + l)
        xc = _rand(nc, c.nrhs, 7 + l)
        P = c.H.P[l]
        assert np.abs(p.restrict(l, xf) - (P.T @ xf.T).T).max() <= 1e-14 * np.abs(xf).max() * 8
        assert np.abs(p.prolong(l, xc) - (P @ xc.T).T).max() <= 1e-15 * np.abs(xc).max() * 8


def test_coarse_solve(case):
    c, p = case
    lc = c.nlevels - 1
    n = p.level_dims(lc)[1]
    b = _rand(n, c.nrhs, 9)
    b[:, c.H.mask[lc].astype(bool)] = 0.0
    x = p.coarse_solve(b)
    ref = np.linalg.solve(c.H.A[lc].toarray(), b.T).T
    assert rel(x, ref) <= 1e-9


def test_vcycle_matches_algorithm1(case):
    from oracle import multigrid
    c, p = case
    r = _rand(p.ndof, c.nrhs, 13)
    r[:, c.mask.astype(bool)] = 0.0
    z = p.precondition(r)
    for l in range(c.nrhs):
        ref = multigrid.vcycle(c.H, r[l], omega=c.omega)
        assert rel(z[l], ref) <= 1e-9


def test_mixed_precision_operators():
    need_gpu()
    c = Case("cantilever", (8, 4, 4), 1, 2, 3, 2, seed=3, precision="mixed")
    p = c.problem()
    p.set_densities(c.rho)
    x = _rand(p.ndof, 2, 4)
    # the outer CG operator stays FP64
    assert np.abs(p.apply(0, x) - (c.H.A[0] @ x.T).T).max() <= 1e-13 * np.abs(c.H.A[0] @ x.T).max()
    # the V-cycle copies are FP32: relative error at single-precision level
    for l in range(c.nlevels):
        n = p.level_dims(l)[1]
        xl = _rand(n, 2, 20 + l)
        ref = (c.H.A[l] @ xl.T).T
        assert np.abs(p.apply(l, xl, "mixed") - ref).max() <= 5e-6 * np.abs(ref).max()
    p.close()


def test_mixed_precision_matrix_free_fine_operator():
    need_gpu()
    from oracle import multigrid
    c = Case("cantilever", (6, 2, 2), 1, 1, 2, 4, seed=21, precision="mixed")
    p = c.problem()
    p.set_densities(c.rho)
    for l in range(c.nlevels):
        n = p.level_dims(l)[1]
        xl = _rand(n, 4, 30 + l)
        ref = (c.H.A[l] @ xl.T).T
        assert np.abs(p.apply(l, xl, "mixed") - ref).max() <= 5e-6 * np.abs(ref).max()
    r = _rand(p.ndof, 4, 40)
    r[:, c.mask.astype(bool)] = 0.0
    z = p.precondition(r)
    for l in range(4):
        assert rel(z[l], multigrid.vcycle(c.H, r[l], omega=c.omega)) <= 1e-4
    p.close()


# Matrix-free trilinear apply (wave tiles of 7 x 7 owned nodes) on lattices
# with ragged tiles in x and y, many plane chunks, long rows, several load
# cases and a single element.
MF_LATTICES = [
    ("cantilever", (40, 12, 10), 2, 1),   # 41 x 13 nodes per plane: ragged tiles
    ("torsion", (24, 20, 30), 2, 3),      # 21 = 3 x 7 node rows: whole tiles, 3 load cases
    ("cantilever", (40, 12, 100), 3, 1),  # 101 node planes
    ("mbb", (130, 4, 6), 2, 2),           # 131-node rows
    ("cantilever", (254, 2, 4), 2, 1),    # 255-node rows
    ("cantilever", (256, 2, 2), 2, 4),    # 257-node rows, 4 load cases
    ("cantilever", (6, 6, 6), 1, 1),      # one tile
    ("cantilever", (1, 1, 1), 1, 1),      # one element
]


@pytest.mark.parametrize("kind,nel,nlev,nrhs", MF_LATTICES,
                         ids=[f"{k}-{'x'.join(map(str, n))}-r{r}" for k, n, _, r in MF_LATTICES])
def test_matrix_free_apply_lattices(kind, nel, nlev, nrhs):
    need_gpu()
    for prec, tol in (("fp64", 1e-13), ("mixed", 5e-6)):
        c = Case(kind, nel, 1, 1, nlev, nrhs, field="uniform", seed=17, precision=prec)
        p = c.problem()
        p.set_densities(c.rho)
        x = _rand(p.ndof, nrhs, 3)
        ref = (c.H.A[0] @ x.T).T
        scale = np.abs(ref).max()
        assert np.abs(p.apply(0, x) - ref).max() <= 1e-13 * scale
        if prec == "mixed":
            assert np.abs(p.apply(0, x, "mixed") - ref).max() <= tol * scale
        p.close()


# Lattices on which the chunk height chosen for the chip's occupancy is
# more than one plane (FP64 / FP32 chunks: 2 / 1, 3 / 2, 3 with a 2-plane
# last chunk / 2, 3 with a whole last chunk / 2): odd and even layer counts
# per wave and ragged last chunks.  Reference: the oracle's element-by-
# element K u with the supports applied.
MF_CHUNK_LATTICES = [((64, 32, 64), 5), ((96, 48, 48), 5), ((96, 64, 40), 4), ((80, 40, 80), 4)]


@pytest.mark.parametrize("nel,nlev", MF_CHUNK_LATTICES,
                         ids=["x".join(map(str, n)) for n, _ in MF_CHUNK_LATTICES])
def test_matrix_free_apply_chunk_heights(nel, nlev):
    need_gpu()
    import workloads as W
    from oracle import assemble, fem
    from paper_2311_05595_amd import api
    mask, f = W.make_problem("cantilever", *nel, 1, 2)
    rho = np.random.default_rng(41).uniform(0.05, 1.0, nel[::-1])
    x = _rand(mask.size, 2, 43)
    x[:, mask.astype(bool)] = 0.0
    ref = assemble.apply(rho, nel, 1, 1, fem.sub_element_matrices(1, 1), x, **MAT)
    ref[:, mask.astype(bool)] = 0.0
    scale = np.abs(ref).max()
    for prec, tol in (("fp64", 1e-13), ("mixed", 5e-6)):
        print(f"[mf chunks] {nel} {prec}", flush=True)
        p = api.Problem(nel, mask, f, order=1, nsub=1, nlevels=nlev, precision=prec)
        p.set_densities(rho.ravel())
        assert np.abs(p.apply(0, x) - ref).max() <= 1e-13 * scale
        if prec == "mixed":
            assert np.abs(p.apply(0, x, "mixed") - ref).max() <= tol * scale
        p.close()


def test_vcycle_matches_algorithm1_multi_range():
    """The V-cycle (its fused finest-level epilogues included) on a lattice of
    several node ranges and plane chunks."""
    need_gpu()
    from oracle import multigrid
    c = Case("cantilever", (40, 12, 10), 1, 1, 2, 2, seed=23)
    p = c.problem()
    p.set_densities(c.rho)
    r = _rand(p.ndof, 2, 29)
    r[:, c.mask.astype(bool)] = 0.0
    z = p.precondition(r)
    for l in range(2):
        assert rel(z[l], multigrid.vcycle(c.H, r[l], omega=c.omega)) <= 1e-9
    p.close()
