"""Pins of the oracle's serendipity elements (Sec. 2.1), quadratic (20
nodes) and cubic (32 nodes): Kronecker property, the 20 or 32 monomials of
their spaces reproduced (and x^2 y^2 not), rank 3 n_e - 6 = 54 and 90 (the
rank rule of Sec. 3.5), rigid-body null space, the uniform-strain energy,
the sub-element matrices summing to the element matrix and the
position-dependent energy of every sub-box."""

import itertools

import numpy as np
import pytest

from oracle import fem

S2 = [a for a in range(27) if fem.serendipity_node(a)]
COORD = np.array([(a % 3 - 1, (a // 3) % 3 - 1, a // 9 - 1) for a in range(27)], dtype=float)


def test_twenty_nodes_and_kronecker():
    assert len(S2) == 20
    for a in S2:
        N, _ = fem.serendipity_shapes(*COORD[a])
        assert np.allclose(N[S2], np.eye(27)[a][S2], atol=1e-15)


def _space():
    """The monomials x^i y^j z^k of superlinear degree <= 2 (the total degree
    less the number of variables of exponent 1): the 20 terms of the
    quadratic serendipity space."""
    mons = [(i, j, k) for i, j, k in itertools.product(range(5), repeat=3)
            if i + j + k - [i, j, k].count(1) <= 2]
    return sorted(mons)


def test_reproduces_its_monomials():
    mons = _space()
    assert len(mons) == 20
    rng = np.random.default_rng(0)
    for _ in range(20):
        p = rng.uniform(-1, 1, 3)
        N, G = fem.serendipity_shapes(*p)
        assert abs(N.sum() - 1.0) < 1e-14
        for (i, j, k) in mons:
            vals = COORD[:, 0] ** i * COORD[:, 1] ** j * COORD[:, 2] ** k
            assert abs(N @ vals - p[0] ** i * p[1] ** j * p[2] ** k) < 1e-13
            # gradients too (d/dx of x^i y^j z^k)
            gx = i * p[0] ** max(i - 1, 0) * p[1] ** j * p[2] ** k
            assert abs(G[:, 0] @ vals - gx) < 1e-13
    # x^2 y^2 is outside the space (the 27-node Lagrange element has it)
    p = np.array([0.3, -0.4, 0.2])
    N, _ = fem.serendipity_shapes(*p)
    vals = COORD[:, 0] ** 2 * COORD[:, 1] ** 2
    assert abs(N @ vals - p[0] ** 2 * p[1] ** 2) > 1e-3


def test_element_matrix_rank_and_rigid_modes():
    K = fem.element_matrix(2, family="serendipity")
    dofs = np.array([3 * a + c for a in S2 for c in range(3)])
    assert np.abs(K - K.T).max() < 1e-14
    others = np.setdiff1d(np.arange(81), dofs)
    assert np.all(K[others] == 0.0) and np.all(K[:, others] == 0.0)
    Ks = K[np.ix_(dofs, dofs)]
    ev = np.linalg.eigvalsh(Ks)
    assert int((ev > 1e-10 * ev.max()).sum()) == 3 * 20 - 6
    R = fem.rigid_body_modes(fem.local_node_coords(2))
    assert np.abs(K @ R.T).max() < 1e-12


@pytest.mark.parametrize("strain", [0, 3, 5])
def test_uniform_strain_energy_and_subelements(strain):
    """u = eps x for a unit strain state: u^T K u = eps^T D eps (unit
    volume); the 8 sub-element matrices sum to the element matrix."""
    K = fem.element_matrix(2, family="serendipity")
    X = fem.local_node_coords(2)
    e = np.zeros(6)
    e[strain] = 1.0
    # displacement gradient from the Voigt strain (engineering shears split)
    F = np.array([[e[0], e[3] / 2, e[5] / 2], [e[3] / 2, e[1], e[4] / 2],
                  [e[5] / 2, e[4] / 2, e[2]]])
    u = (X @ F.T).reshape(-1)
    D = fem.elasticity_matrix()
    assert u @ K @ u == pytest.approx(e @ D @ e, rel=1e-12)
    Ksub = fem.sub_element_matrices(2, 2, family="serendipity")
    assert np.abs(Ksub.sum(axis=0) - K).max() < 1e-13


def test_dof_mask_marks_face_and_body_centres():
    m = fem.serendipity_dof_mask((2, 1, 1))
    nodes = m[::3].reshape(3, 3, 5)
    # per element 6 face centres + 1 body centre; the two elements share one face
    assert nodes.sum() == 2 * 7 - 1


# ---------------------------------------------------------------- cubic (32 nodes)
S3 = [a for a in range(64) if fem.serendipity_node(a, 3)]
COORD3 = np.array([[-1.0 + 2.0 * q / 3.0 for q in (a % 4, (a // 4) % 4, a // 16)]
                   for a in range(64)])


def _space3():
    """Monomials of superlinear degree <= 3: the 32 terms of the cubic
    serendipity space (all of total degree <= 3, and x^3 y, x y^3, x^3 z,
    x z^3, y^3 z, y z^3, x^3 y z, x y^3 z, x y z^3)."""
    return sorted((i, j, k) for i, j, k in itertools.product(range(5), repeat=3)
                  if i + j + k - [i, j, k].count(1) <= 3)


def test_thirty_two_nodes_and_kronecker():
    assert len(S3) == 32
    # vertices and the two third-points of each of the 12 edges
    assert sum(all(abs(c) == 1.0 for c in COORD3[a]) for a in S3) == 8
    for a in S3:
        N, _ = fem.serendipity_shapes(*COORD3[a], order=3)
        assert np.abs(N[S3] - np.eye(64)[a][S3]).max() < 1e-15


def test_cubic_reproduces_its_monomials():
    mons = _space3()
    assert len(mons) == 32
    rng = np.random.default_rng(1)
    for _ in range(20):
        p = rng.uniform(-1, 1, 3)
        N, G = fem.serendipity_shapes(*p, order=3)
        assert abs(N.sum() - 1.0) < 1e-14
        for (i, j, k) in mons:
            vals = COORD3[:, 0] ** i * COORD3[:, 1] ** j * COORD3[:, 2] ** k
            assert abs(N @ vals - p[0] ** i * p[1] ** j * p[2] ** k) < 1e-13
            grad = (i * p[0] ** max(i - 1, 0) * p[1] ** j * p[2] ** k,
                    j * p[0] ** i * p[1] ** max(j - 1, 0) * p[2] ** k,
                    k * p[0] ** i * p[1] ** j * p[2] ** max(k - 1, 0))
            for d in range(3):
                assert abs(G[:, d] @ vals - grad[d]) < 1e-12
    # x^2 y^2 is outside the space (the 64-node Lagrange element has it)
    p = np.array([0.3, -0.4, 0.2])
    N, _ = fem.serendipity_shapes(*p, order=3)
    vals = COORD3[:, 0] ** 2 * COORD3[:, 1] ** 2
    assert abs(N @ vals - p[0] ** 2 * p[1] ** 2) > 1e-3


def test_cubic_element_matrix_rank_and_rigid_modes():
    K = fem.element_matrix(3, family="serendipity")
    dofs = np.array([3 * a + c for a in S3 for c in range(3)])
    assert np.abs(K - K.T).max() < 1e-14
    others = np.setdiff1d(np.arange(192), dofs)
    assert np.all(K[others] == 0.0) and np.all(K[:, others] == 0.0)
    ev = np.linalg.eigvalsh(K[np.ix_(dofs, dofs)])
    assert int((ev > 1e-10 * ev.max()).sum()) == 3 * 32 - 6
    R = fem.rigid_body_modes(fem.local_node_coords(3))
    assert np.abs(K @ R.T).max() < 1e-12


@pytest.mark.parametrize("strain", [0, 1, 3, 5])
def test_cubic_uniform_strain_energy_and_subelements(strain):
    K = fem.element_matrix(3, family="serendipity")
    X = fem.local_node_coords(3)
    e = np.zeros(6)
    e[strain] = 1.0
    F = np.array([[e[0], e[3] / 2, e[5] / 2], [e[3] / 2, e[1], e[4] / 2],
                  [e[5] / 2, e[4] / 2, e[2]]])
    u = (X @ F.T).reshape(-1)
    D = fem.elasticity_matrix()
    assert u @ K @ u == pytest.approx(e @ D @ e, rel=1e-12)
    Ksub = fem.sub_element_matrices(3, 2, family="serendipity")
    assert np.abs(Ksub.sum(axis=0) - K).max() < 1e-13


@pytest.mark.parametrize("order", [2, 3])
def test_sub_box_energies_of_a_bilinear_field(order):
    """u_x = x y lies in both serendipity spaces; its energy on the sub-box
    [lo, hi] of the unit element is 1/2 of the integral of (M y^2 + G x^2)
    (M = lambda + 2 mu, G = mu), which pins every sub-matrix to its box."""
    nu = 0.3
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    G = 1.0 / (2 * (1 + nu))
    M = lam + 2 * G
    X = fem.local_node_coords(order)
    u = np.zeros(3 * X.shape[0])
    u[0::3] = X[:, 0] * X[:, 1]
    n = 2
    Ks = fem.sub_element_matrices(order, n, nu, family="serendipity")
    for sz in range(n):
        for sy in range(n):
            for sx in range(n):
                lo = np.array([sx, sy, sz]) / n
                hi = lo + 1.0 / n
                vol = np.prod(hi - lo)
                iy2 = vol / (hi[1] - lo[1]) * (hi[1] ** 3 - lo[1] ** 3) / 3.0
                ix2 = vol / (hi[0] - lo[0]) * (hi[0] ** 3 - lo[0] ** 3) / 3.0
                ref = 0.5 * (M * iy2 + G * ix2)
                got = 0.5 * u @ Ks[sx + n * (sy + n * sz)] @ u
                assert abs(got - ref) < 1e-14


def test_cubic_dof_mask_marks_face_and_body_interiors():
    m = fem.serendipity_dof_mask((2, 1, 1), 3)
    nodes = m[::3].reshape(4, 4, 7)
    # per element 24 face-interior + 8 body-interior nodes; the shared face
    # has 4 interior nodes
    assert nodes.sum() == 2 * 32 - 4
    # a lattice node is kept iff at most one index is off the vertex lattice
    k, j, i = np.meshgrid(np.arange(4), np.arange(4), np.arange(7), indexing="ij")
    inner = (i % 3 != 0).astype(int) + (j % 3 != 0) + (k % 3 != 0)
    assert np.array_equal(nodes.astype(bool), inner >= 2)
