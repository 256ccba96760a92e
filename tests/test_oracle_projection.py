"""Pins of the oracle's design-variable projection / density filter (Sec. 2.2
eq. (4), Sec. 3.2 eq. (5)) and its chain rule (Sec. 3.4)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import assemble, fem, projection as P, solve

MAT = dict(E0=1.0, Emin=1e-9, penal=3.0)


def _brute_force_matrix(nel, n, d, rmin):
    """All pairs from floating-point cell centres, the ball test on the
    Euclidean distance itself, weights exp(-dist^2/(2 s^2))/(2 pi s), s = rmin/3,
    rows divided by their sums (radii below are chosen away from ties)."""
    def centres(m):
        z, y, x = np.meshgrid(*(np.arange(m * nel[a]) for a in (2, 1, 0)), indexing="ij")
        return np.stack([(x.ravel() + 0.5) / m, (y.ravel() + 0.5) / m, (z.ravel() + 0.5) / m], 1)
    cr, cx = centres(n), centres(d)
    dist = np.sqrt(((cr[:, None, :] - cx[None, :, :]) ** 2).sum(-1))
    s = rmin / 3.0
    om = np.where(dist <= rmin, np.exp(-dist ** 2 / (2 * s * s)) / (2 * np.pi * s), 0.0)
    return om / om.sum(1, keepdims=True)


@pytest.mark.parametrize("nel,n,d,rmin", [
    ((3, 2, 2), 1, 1, 1.3), ((2, 2, 1), 2, 1, 0.77), ((2, 1, 1), 4, 2, 0.61),
    ((2, 2, 2), 2, 2, 1.13), ((1, 2, 1), 3, 1, 0.9), ((2, 1, 1), 2, 4, 0.7)])
def test_all_pairs_brute_force(nel, n, d, rmin):
    Wb = _brute_force_matrix(nel, n, d, rmin)
    Wo = P.projection_matrix(nel, n, d, rmin).toarray()
    assert Wo.shape == Wb.shape
    assert np.abs(Wo - Wb).max() <= 1e-14


@pytest.mark.parametrize("nel,n,d,rmin", [((4, 3, 2), 4, 2, 0.6), ((3, 3, 3), 1, 1, 2.0),
                                          ((2, 2, 2), 4, 2, 1.5)])
def test_partition_of_unity(nel, n, d, rmin):
    """Each density is a weighted average: W 1 = 1, so a constant design is
    projected onto the same constant."""
    Wm = P.projection_matrix(nel, n, d, rmin)
    assert np.abs(np.asarray(Wm.sum(axis=1)).ravel() - 1.0).max() <= 1e-15
    assert Wm.min() >= 0.0
    x = np.full(Wm.shape[1], 0.37)
    assert np.abs(Wm @ x - 0.37).max() <= 1e-15


def test_two_cells_closed_form():
    """n = d = 1, two unit cells side by side, rmin = 1: the neighbour lies
    exactly on the ball's boundary (dist = rmin, inside) with weight
    exp(-1 / (2 (1/3)^2)) = e^{-4.5} relative to the cell itself."""
    e = math.exp(-4.5)
    x = np.array([1.0, 0.0])
    rho = P.project(x, (2, 1, 1), 1, 1, 1.0)
    assert abs(rho[0] - 1.0 / (1.0 + e)) <= 1e-15
    assert abs(rho[1] - e / (1.0 + e)) <= 1e-15
    # three cells: the middle one averages both neighbours
    x3 = np.array([0.2, 0.5, 0.9])
    rho3 = P.project(x3, (3, 1, 1), 1, 1, 1.0)
    assert abs(rho3[1] - (e * 0.2 + 0.5 + e * 0.9) / (1 + 2 * e)) <= 1e-15
    # just below the boundary the neighbours drop out: the identity
    assert np.abs(P.project(x3, (3, 1, 1), 1, 1, 0.999) - x3).max() == 0.0


def test_identity_when_radius_below_spacing():
    """d = n and rmin below the cell spacing 1/n: each ball holds its own cell."""
    rng = np.random.default_rng(4)
    for n in (1, 2, 4):
        nel = (2, 2, 1)
        x = rng.random(P.lattice_shape(nel, n)).ravel()
        assert np.array_equal(P.project(x, nel, n, n, 0.9 / n), x)


def test_single_entries_match_matrix():
    rng = np.random.default_rng(5)
    nel, n, d, rmin = (3, 2, 2), 4, 2, 1.5
    Wm = P.projection_matrix(nel, n, d, rmin)
    x = rng.random(Wm.shape[1])
    g = rng.standard_normal(Wm.shape[0])
    rho, gx = Wm @ x, Wm.T @ g
    Sr, Sx = P.lattice_shape(nel, n), P.lattice_shape(nel, d)
    for flat in rng.choice(Wm.shape[0], 12, replace=False):
        i3 = (flat % Sr[2], (flat // Sr[2]) % Sr[1], flat // (Sr[2] * Sr[1]))
        assert abs(P.project_at(x, i3, nel, n, d, rmin) - rho[flat]) <= 1e-14
    for flat in rng.choice(Wm.shape[1], 6, replace=False):
        k3 = (flat % Sx[2], (flat // Sx[2]) % Sx[1], flat // (Sx[2] * Sx[1]))
        assert abs(P.project_transpose_at(g, k3, nel, n, d, rmin) - gx[flat]) <= 1e-12 * (
            1 + abs(gx[flat]))


def test_rejects_empty_ball():
    # n = 4, d = 2: the nearest design centre is 0.125 * sqrt(3) away
    with pytest.raises(ValueError):
        P.projection_matrix((1, 1, 1), 4, 2, 0.2)


def test_chain_rule_finite_differences():
    """df/dx = W^T dc (Sec. 3.4) for f(x) = c(rho(x)), against central
    differences of the oracle's own solve along seeded directions."""
    nel, n, d, rmin = (3, 1, 1), 2, 1, 0.9
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    Ks = fem.sub_element_matrices(1, n)
    rng = np.random.default_rng(11)
    x = 0.3 + 0.5 * rng.random(int(np.prod(P.lattice_shape(nel, d))))
    Wm = P.projection_matrix(nel, n, d, rmin)

    def comp(xv):
        rho = (Wm @ xv).reshape(P.lattice_shape(nel, n))
        _, _, c, dc = solve.solve_problem(rho, mask, f, nel, 1, n, Ks, **MAT)
        return c.sum(), dc

    c0, dc = comp(x)
    gx = P.project_transpose(dc, nel, n, d, rmin)
    h = 1e-6
    for s in range(3):
        v = rng.choice([-1.0, 1.0], x.size)
        fd = (comp(x + h * v)[0] - comp(x - h * v)[0]) / (2 * h)
        assert abs(fd - gx @ v) <= 1e-6 * abs(fd)


def test_volume_gradient_sums():
    """sum_k (W^T v)_k = sum_i v_i sum_k W_ik = sum_i v_i, the domain's volume
    (rows of W sum to one); every design cell has a positive share."""
    nel, n, d, rmin = (3, 2, 2), 4, 2, 0.6
    gv = P.volume_gradient(nel, n, d, rmin)
    assert abs(gv.sum() - np.prod(nel)) <= 1e-12
    assert gv.min() > 0.0
