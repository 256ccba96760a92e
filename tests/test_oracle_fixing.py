"""Pins of the oracle's choice of fixed variables (Sec. 6.1): hand-counted
cases, the surrounded rule against scipy's binary erosion, the node rule
against a closed form over padded element lattices, and the paper's claim
that the suppressed void DOFs barely change the compliance."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import fem, solve
from oracle import fixing as F
import workloads as W


def _block_case(nel=(6, 4, 4), n=2, d=1, split=3, left=0.0, right=0.5):
    """Densities `left` for the elements with ex < split, `right` beyond."""
    nelx, nely, nelz = nel
    ex = np.arange(n * nelx) // n
    rho = np.broadcast_to(np.where(ex < split, left, right), (n * nelz, n * nely, n * nelx)).copy()
    grad = np.zeros((d * nelz, d * nely, d * nelx))
    return rho, grad


def test_void_block_by_hand():
    """Void for ex < 3 on a 6x4x4 mesh: ex = 2 touches mixed elements, so 2 x 4
    x 4 = 32 elements are fixed; the Q1 nodes with x index 0 or 1 (2 x 5 x 5 =
    50) and the Q2 nodes with x index 0..3 (4 x 9 x 9 = 324) touch only them."""
    nel, n, d = (6, 4, 4), 2, 1
    rho, grad = _block_case(nel, n, d)
    kind = F.classify(rho, grad, nel, n, d)
    assert np.all(kind[:, :, :3] == F.VOID) and np.all(kind[:, :, 3:] == F.MIXED)
    fk = F.surrounded(kind)
    assert np.all(fk[:, :, :2] == F.VOID) and np.all(fk[:, :, 2:] == F.MIXED)
    assert (fk == F.VOID).sum() == 32
    n1 = F.suppressed_nodes(fk, 1)
    assert n1.sum() == 50 and np.all(n1[:, :, :2] == 1)
    n2 = F.suppressed_nodes(fk, 2)
    assert n2.sum() == 324 and np.all(n2[:, :, :4] == 1)
    fd = F.fixed_design(fk, d)
    assert fd.sum() == 32 and np.all(fd[:, :, :2] == 1)


def test_gradient_vetoes_and_solid_block():
    """A gradient component below -eps in element (0,0,0) makes it mixed and
    unfixes the 8 elements around that corner (32 - 8 = 24 fixed); a solid
    block (rho = 0.95) for ex >= 3 fixes ex = 4, 5 as solid, and the design
    variables (d = 2) of both blocks."""
    nel, n, d = (6, 4, 4), 2, 2
    rho, grad = _block_case(nel, n, d, left=0.0, right=0.95)
    grad[0, 0, 0] = -1e-3
    kind = F.classify(rho, grad, nel, n, d)
    assert kind[0, 0, 0] == F.MIXED
    fk = F.surrounded(kind)
    assert (fk == F.VOID).sum() == 24
    assert (fk == F.SOLID).sum() == 32 and np.all(fk[:, :, 4:] == F.SOLID)
    assert F.fixed_design(fk, d).sum() == (24 + 32) * d ** 3
    # a gradient above eps vetoes a solid element the same way
    grad[:, :, -1] = 1e-3
    fk2 = F.surrounded(F.classify(rho, grad, nel, n, d))
    assert (fk2 == F.SOLID).sum() == 0
    # thresholds are inclusive
    rho_edge = np.full((n * 4, n * 4, n * 6), 1e-6)
    assert np.all(F.classify(rho_edge, np.full((d * 4, d * 4, d * 6), -1e-6), nel, n, d) == F.VOID)


@pytest.mark.parametrize("seed", range(4))
def test_surrounded_is_erosion(seed):
    rng = np.random.default_rng(seed)
    shape = (5, 7, 9)
    blobs = ndimage.gaussian_filter(rng.random(shape), 2.0)
    lo, hi = np.quantile(blobs, [0.35, 0.65])
    kind = np.where(blobs < lo, F.VOID, np.where(blobs > hi, F.SOLID, F.MIXED)).astype(np.uint8)
    fk = F.surrounded(kind)
    for k in (F.VOID, F.SOLID):
        # outside the domain counts as "same kind" (neighbours there do not exist)
        er = ndimage.binary_erosion(kind == k, structure=np.ones((3, 3, 3)), border_value=1)
        assert np.array_equal(fk == k, er & (kind == k))
    assert (fk != F.MIXED).sum() > 0


@pytest.mark.parametrize("order,seed", [(1, 0), (2, 1), (1, 2), (2, 3), (3, 4)])
def test_node_rule_closed_form(order, seed):
    """A node's elements along one axis are (i - 1) // p and i // p (one
    element when i is not a multiple of p): padding the fixed-void lattice
    with True and taking the AND over the 8 index combinations gives the
    same nodes."""
    rng = np.random.default_rng(seed)
    blobs = ndimage.gaussian_filter(rng.random((4, 5, 6)), 1.5)
    fk = np.where(blobs < np.quantile(blobs, 0.6), F.VOID, F.MIXED).astype(np.uint8)
    p = order
    pad = np.pad(fk == F.VOID, 1, constant_values=True)
    idx = [np.arange(p * s + 1) for s in fk.shape]
    lo = [(i - 1) // p + 1 for i in idx]
    hi = [i // p + 1 for i in idx]
    out = np.ones(tuple(len(i) for i in idx), dtype=bool)
    for a in (lo[0], hi[0]):
        for b in (lo[1], hi[1]):
            for c in (lo[2], hi[2]):
                out &= pad[np.ix_(a, b, c)]
    assert np.array_equal(F.suppressed_nodes(fk, order), out.astype(np.uint8))


@pytest.mark.parametrize("order", [1, 2, 3])
def test_suppressed_void_dofs_barely_change_compliance(order):
    """Cantilever 8x6x4 with a void block (rho = 1e-7) in the top layers
    ex = 2..6, ey = 3..5: fixing the DOFs of the nodes inside the fixed void
    region changes the compliance by less than 1e-6 of itself (E_min = 1e-9,
    Sec. 6.1)."""
    nel, n = (8, 6, 4), 1
    rho = np.ones((4, 6, 8))
    rho[:, 3:, 2:7] = 1e-7
    kind = F.classify(rho, np.zeros_like(rho), nel, n, 1)
    fk = F.surrounded(kind)
    nodes = F.suppressed_nodes(fk, order)
    assert nodes.sum() > 0
    mask, f = W.make_problem("cantilever", *nel, order, 1)
    Ks = fem.sub_element_matrices(order, n)
    mat = dict(E0=1.0, Emin=1e-9, penal=3.0)
    _, _, c, _ = solve.solve_problem(rho, mask, f, nel, order, n, Ks, **mat)
    m2 = F.dof_mask(mask, nodes)
    assert m2.sum() > mask.sum()
    _, u2, c2, _ = solve.solve_problem(rho, m2, f, nel, order, n, Ks, **mat)
    assert abs(c2.sum() - c.sum()) <= 1e-6 * c.sum()
