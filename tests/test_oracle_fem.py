"""Pins of the oracle's element matrices against facts fixed by the paper and
by continuum mechanics (not against the oracle's own formulas)."""

import os

import numpy as np
import pytest

from oracle import fem

E, NU = 1.0, 0.3
# textbook moduli of isotropic elasticity
G = E / (2 * (1 + NU))                       # shear modulus
M = E * (1 - NU) / ((1 + NU) * (1 - 2 * NU))  # P-wave (constrained) modulus
KB = E / (3 * (1 - 2 * NU))                   # bulk modulus


def _rank_table(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "table1_rank_bounds.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("order", [1, 2, 3])
def test_rank_matches_table1(order, golden_dir):
    """Sec. 3.5 Table 1: rank(K^(e)) = 3 n_e - 6 (18, 75, 186)."""
    table = {deg: (nodes, rank) for deg, nodes, rank in _rank_table(golden_dir)}
    K = fem.element_matrix(order, NU)
    nodes, rank = table[order]
    assert K.shape == (3 * nodes, 3 * nodes)
    assert np.linalg.matrix_rank(K, tol=1e-10 * np.abs(K).max()) == rank


@pytest.mark.parametrize("order", [1, 2, 3])
def test_symmetric_and_rigid_modes(order):
    K = fem.element_matrix(order, NU)
    assert np.abs(K - K.T).max() < 1e-15
    R = fem.rigid_body_modes(fem.local_node_coords(order))
    assert np.abs(K @ R.T).max() < 1e-13
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-13  # positive semi-definite


def test_q1_diagonal_closed_form():
    """Unit cube, trilinear: the integral of (dN_a/dx)^2 is 1 * 1/3 * 1/3, so
    K_(a,x),(a,x) = (M + 2G)/9."""
    K = fem.element_matrix(1, NU)
    assert abs(K[0, 0] - (M + 2 * G) / 9.0) < 1e-15
    assert np.allclose(np.diag(K), (M + 2 * G) / 9.0, rtol=0, atol=1e-15)


def _linear_field(coords, grad):
    """Nodal displacements of u(x) = grad @ x at the given coordinates."""
    return (coords @ grad.T).ravel()


STRAINS = {
    # name: (displacement gradient, energy density of that uniform strain)
    "uniaxial_x": (np.diag([1.0, 0, 0]), 0.5 * M),
    "uniaxial_z": (np.diag([0, 0, 1.0]), 0.5 * M),
    "hydrostatic": (np.eye(3), 4.5 * KB),
    "simple_shear_xy": (np.array([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]]), 0.5 * G),
    "simple_shear_zy": (np.array([[0, 0, 0], [0, 0, 0], [0, 1.0, 0]]), 0.5 * G),
    "rotation": (np.array([[0, -1.0, 0], [1.0, 0, 0], [0, 0, 0]]), 0.0),
}


@pytest.mark.parametrize("order", [1, 2, 3])
@pytest.mark.parametrize("name", list(STRAINS))
def test_uniform_strain_energy(order, name):
    """A linear displacement field has uniform strain; Lagrange elements
    reproduce it exactly, so 1/2 u^T K u equals (volume) * energy density."""
    grad, wdens = STRAINS[name]
    u = _linear_field(fem.local_node_coords(order), grad)
    K = fem.element_matrix(order, NU)
    assert abs(0.5 * u @ K @ u - wdens) < 1e-13


@pytest.mark.parametrize("order,nsub", [(1, 2), (1, 3), (1, 4), (2, 2), (2, 4), (3, 2)])
def test_sub_elements_split_the_integral(order, nsub):
    """Sec. 3.3: the element integral is the sum of the n^3 sub-box integrals,
    and each sub-box carries 1/n^3 of a uniform-strain energy (which fixes the
    sub-interval length in local coordinates)."""
    Ks = fem.sub_element_matrices(order, nsub, NU)
    K = fem.element_matrix(order, NU)
    assert Ks.shape[0] == nsub ** 3
    assert np.abs(Ks.sum(0) - K).max() < 1e-14 * max(1.0, np.abs(K).max()) * nsub ** 3
    for name in ("uniaxial_x", "hydrostatic", "simple_shear_xy"):
        grad, wdens = STRAINS[name]
        u = _linear_field(fem.local_node_coords(order), grad)
        e = 0.5 * np.einsum("a,sab,b->s", u, Ks, u)
        assert np.abs(e - wdens / nsub ** 3).max() < 1e-14


def test_q1_n4_sub_matrices_span_23_dimensions():
    """Design fact used by the HIP path's choice of storage: the 64 Q1
    sub-element matrices are not independent."""
    Ks = fem.sub_element_matrices(1, 4, NU)
    assert np.linalg.matrix_rank(Ks.reshape(64, -1), tol=1e-12) == 23


def test_scaling_with_element_size():
    """3-D stiffness scales linearly with the element edge: a cube of edge 2
    has twice the matrix of the unit cube."""
    K1 = fem.sub_element_matrices(1, 1, NU, half=(0.5, 0.5, 0.5))[0]
    K2 = fem.sub_element_matrices(1, 1, NU, half=(1.0, 1.0, 1.0))[0]
    assert np.abs(K2 - 2 * K1).max() < 1e-14


# Bilinear displacement fields whose energy density depends on position, one
# per pair of axes: u = (xy, 0, 0) has eps_xx = y and gamma_xy = x, so its
# energy density is (M y^2 + G x^2)/2; (0, yz, 0) and (0, 0, zx) are its
# cyclic images.  M != G, so swapping two axes of a sub-box changes its energy.
def _bilinear_field(coords, comp):
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    u = np.zeros((coords.shape[0], 3))
    u[:, comp] = (x * y, y * z, z * x)[comp]
    return u.ravel()


def _box_energy(comp, lo, hi):
    """Integral of the field's energy density over the box [lo, hi]: with
    (a, b) the axes of the field's two factors (the strain along a is the b
    coordinate, the shear gamma_ab is the a coordinate), the density is
    (M t_b^2 + G t_a^2)/2, integrated in closed form."""
    a, b = ((0, 1), (1, 2), (2, 0))[comp]
    vol = np.prod(np.subtract(hi, lo))

    def sq(ax):  # integral of t_ax^2 over the box
        return vol / (hi[ax] - lo[ax]) * (hi[ax] ** 3 - lo[ax] ** 3) / 3.0

    return 0.5 * (M * sq(b) + G * sq(a))


@pytest.mark.parametrize("order,nsub", [(1, 2), (1, 4), (2, 2), (2, 4), (3, 2)])
def test_sub_element_placement(order, nsub):
    """Sec. 3.3 eq. (7): K^(e_i) integrates over sub-box i = sx + n (sy + n sz),
    which covers [sx/n, (sx+1)/n] x [sy/n, ...] x [sz/n, ...] of the unit
    element.  Position-dependent energies fix each sub-matrix to its box
    (the sub-element sum and uniform strains cannot: they are symmetric
    under permutations of the boxes)."""
    Ks = fem.sub_element_matrices(order, nsub, NU)
    coords = fem.local_node_coords(order)
    for comp in range(3):
        u = _bilinear_field(coords, comp)
        for sz in range(nsub):
            for sy in range(nsub):
                for sx in range(nsub):
                    lo = np.array([sx, sy, sz], dtype=float) / nsub
                    hi = lo + 1.0 / nsub
                    e = 0.5 * u @ Ks[sx + nsub * (sy + nsub * sz)] @ u
                    assert abs(e - _box_energy(comp, lo, hi)) < 1e-14, (comp, sx, sy, sz)


@pytest.mark.parametrize("order,nsub", [(1, 2), (2, 2), (1, 3)])
def test_density_cell_placement(order, nsub):
    """The density lattice (C order [n nelz][n nely][n nelx]) against the
    geometry: with E = rho^p (Emin = 0) and a single solid density cell, the
    assembled energy of a global bilinear field is the closed-form energy of
    that cell's box in the mesh's coordinates (element (ex, ey, ez) at the
    origin (ex, ey, ez), cell (ix, iy, iz) on [ix/n, (ix+1)/n] x ...)."""
    from oracle import assemble

    nel = (3, 2, 2)
    Ks = fem.sub_element_matrices(order, nsub, NU)
    dims = assemble.node_dims(nel, order)
    t = [np.linspace(0.0, nel[d], dims[d]) for d in range(3)]
    Z, Y, X = np.meshgrid(t[2], t[1], t[0], indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    lat = tuple(nsub * v for v in nel)
    rng = np.random.default_rng(11)
    cells = rng.choice(int(np.prod(lat)), size=6, replace=False)
    for cell in cells:
        rho = np.zeros(int(np.prod(lat)))
        rho[cell] = 1.0
        K = assemble.stiffness(rho, nel, order, nsub, Ks, E0=1.0, Emin=0.0)
        ix = cell % lat[0]
        iy = (cell // lat[0]) % lat[1]
        iz = cell // (lat[0] * lat[1])
        lo = np.array([ix, iy, iz], dtype=float) / nsub
        hi = lo + 1.0 / nsub
        for comp in range(3):
            u = _bilinear_field(coords, comp)
            e = 0.5 * u @ (K @ u)
            ref = _box_energy(comp, lo, hi)
            assert abs(e - ref) < 1e-12 * max(1.0, ref), (cell, comp)
