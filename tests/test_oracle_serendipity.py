"""Pins of the oracle's quadratic serendipity element (Sec. 2.1): Kronecker
property, the 20 monomials of its space reproduced (and x^2 y^2 not), rank
3 n_e - 6 = 54 (Table 1), rigid-body null space, the uniform-strain energy,
and the sub-element matrices summing to the element matrix."""

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
