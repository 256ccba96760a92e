"""Element stiffness matrices of rectangular-prism Lagrange elements.

Follows Sec. 2 eq. (1) (K^(e) = E * integral of B^T D B over the element) and
Sec. 3.3 (the integral over [-1,1]^3 split into n^3 sub-boxes, one matrix
K^(e_i) per density sub-element, each computed once for a regular mesh).

* Shape functions: tensor-product Lagrange polynomials on equally spaced
  nodes (degree 1: 8 nodes, 2: 27 nodes, 3: 64 nodes; Sec. 2.1).
  Local node a = ax + (p+1)*(ay + (p+1)*az); local DOF = 3a + c.
* D: isotropic linear elasticity, Voigt order (xx, yy, zz, xy, yz, zx),
  engineering shear strains (textbook; the paper only names "the matrix of
  elastic parameters").
* Geometry: element of size 2l x 2h x 2w with xi = x/l etc., so
  dOmega = l*h*w dxi deta dzeta (Sec. 3.3).  Unit elements: l = h = w = 1/2.
* Sub-box i of the n^3 split covers [-1 + 2a/n, -1 + 2(a+1)/n] per axis in
  local coordinates (the interval length is 2/n in local units, i.e. 1/n of
  the element edge; see the reading listed with the oracle's design notes).
* Quadrature: p+1 Gauss-Legendre points per axis on each sub-box, which is
  exact for the polynomial integrand of degree <= 2p per axis.

* Quadratic serendipity element (20 nodes, Sec. 2.1): the vertices and edge
  midpoints of the 27-node layout, with the textbook shape functions
  (vertex: (1 + xi xi_a)(1 + eta eta_a)(1 + zeta zeta_a)(xi xi_a + eta eta_a
  + zeta zeta_a - 2) / 8; edge midpoint with xi_a = 0: (1 - xi^2)(1 + eta
  eta_a)(1 + zeta zeta_a) / 4, and likewise).  Its matrices keep the 81-DOF
  layout of the 27-node element with zero rows and columns at the 6 face
  centres and the body centre, which a problem then fixes; 3 Gauss points
  per axis integrate them exactly.
* Cubic serendipity element (32 nodes, Sec. 2.1): the vertices and the two
  third-points of every edge of the 64-node layout (local coordinates -1,
  -1/3, 1/3, 1 per axis), with the textbook shape functions (vertex:
  (1 + xi xi_a)(1 + eta eta_a)(1 + zeta zeta_a)(9 (xi^2 + eta^2 + zeta^2)
  - 19) / 64; edge node with |xi_a| = 1/3: 9 (1 - xi^2)(1 + 9 xi xi_a)(1 +
  eta eta_a)(1 + zeta zeta_a) / 64, and likewise).  Its matrices keep the
  192-DOF layout of the 64-node element with zero rows and columns at the 24
  face-interior and 8 body-interior nodes; the shape functions have degree
  3 per axis, so 4 Gauss points per axis integrate the products of their
  gradients exactly.

Pins (tests/test_oracle_fem.py, tests/test_oracle_serendipity.py): symmetry;
rank 3*n_e - 6 (Table 1: 18, 75, 186; the same rule gives 54 and 90 for
the serendipity elements); six rigid-body modes in the null space; the hand-derived diagonal
(D11 + 2G)/9 of the unit Q1 cube; the strain energy of a uniform strain field
equals (volume) * eps^T D eps (closed form per strain state); sum of the
sub-element matrices equals the single-element matrix; each sub-matrix
carries exactly its sub-volume's share of a uniform-strain energy; the
energy of the bilinear fields (xy, 0, 0), (0, yz, 0), (0, 0, zx), which
varies with position, matches the closed form on every sub-box, which fixes
each sub-matrix to its box; and the same closed form over single density
cells of an assembled mesh fixes the density lattice's placement.
"""

import numpy as np


def lagrange_1d(order):
    """Nodes, values and derivatives of the 1-D Lagrange basis on [-1, 1]."""
    nodes = np.linspace(-1.0, 1.0, order + 1)

    def val(xi):
        xi = np.asarray(xi, dtype=np.float64)
        out = np.ones((order + 1,) + xi.shape)
        for k in range(order + 1):
            for m in range(order + 1):
                if m != k:
                    out[k] *= (xi - nodes[m]) / (nodes[k] - nodes[m])
        return out

    def der(xi):
        xi = np.asarray(xi, dtype=np.float64)
        out = np.zeros((order + 1,) + xi.shape)
        for k in range(order + 1):
            for j in range(order + 1):
                if j == k:
                    continue
                term = np.ones(xi.shape) / (nodes[k] - nodes[j])
                for m in range(order + 1):
                    if m != k and m != j:
                        term = term * (xi - nodes[m]) / (nodes[k] - nodes[m])
                out[k] += term
        return out

    return nodes, val, der


def elasticity_matrix(E=1.0, nu=0.3):
    """Isotropic D in Voigt order (xx, yy, zz, xy, yz, zx), engineering shear."""
    c = E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = c * nu
    for i in range(3):
        D[i, i] = c * (1.0 - nu)
    for i in range(3, 6):
        D[i, i] = E / (2.0 * (1.0 + nu))
    return D


def serendipity_node(a, order=2):
    """True for the nodes of the serendipity element of the given degree (2:
    20 nodes, 3: 32 nodes) in the (order+1)^3 Lagrange layout: the vertices
    and the edge nodes, i.e. at most one local index strictly inside the
    element's edge."""
    p1 = order + 1
    idx = (a % p1, (a // p1) % p1, a // (p1 * p1))
    return sum(0 < t < order for t in idx) <= 1


def _serendipity2(xi, eta, zeta):
    N = np.zeros(27)
    G = np.zeros((27, 3))
    for a in range(27):
        if not serendipity_node(a, 2):
            continue
        c = (a % 3 - 1, (a // 3) % 3 - 1, a // 9 - 1)
        t = (xi, eta, zeta)
        if all(ci != 0 for ci in c):
            f = [1.0 + t[d] * c[d] for d in range(3)]
            s = t[0] * c[0] + t[1] * c[1] + t[2] * c[2] - 2.0
            N[a] = f[0] * f[1] * f[2] * s / 8.0
            for d in range(3):
                o = [f[e] for e in range(3) if e != d]
                G[a, d] = c[d] * o[0] * o[1] * (s + f[d]) / 8.0
        else:
            m = [d for d in range(3) if c[d] == 0][0]   # the axis of the midpoint
            f = [1.0 - t[d] ** 2 if d == m else 1.0 + t[d] * c[d] for d in range(3)]
            df = [-2.0 * t[d] if d == m else c[d] for d in range(3)]
            N[a] = f[0] * f[1] * f[2] / 4.0
            G[a, 0] = df[0] * f[1] * f[2] / 4.0
            G[a, 1] = f[0] * df[1] * f[2] / 4.0
            G[a, 2] = f[0] * f[1] * df[2] / 4.0
    return N, G


def _serendipity3(xi, eta, zeta):
    N = np.zeros(64)
    G = np.zeros((64, 3))
    t = (xi, eta, zeta)
    for a in range(64):
        if not serendipity_node(a, 3):
            continue
        c = [-1.0 + 2.0 * q / 3.0 for q in (a % 4, (a // 4) % 4, a // 16)]
        inner = [d for d in range(3) if abs(c[d]) < 1.0]
        if not inner:
            f = [1.0 + t[d] * c[d] for d in range(3)]
            s = 9.0 * (t[0] ** 2 + t[1] ** 2 + t[2] ** 2) - 19.0
            N[a] = f[0] * f[1] * f[2] * s / 64.0
            for d in range(3):
                o = [f[e] for e in range(3) if e != d]
                G[a, d] = o[0] * o[1] * (c[d] * s + f[d] * 18.0 * t[d]) / 64.0
        else:
            m = inner[0]                                  # the axis of the edge
            f = [(1.0 - t[d] ** 2) * (1.0 + 9.0 * c[d] * t[d]) if d == m
                 else 1.0 + t[d] * c[d] for d in range(3)]
            df = [-2.0 * t[d] * (1.0 + 9.0 * c[d] * t[d]) + 9.0 * c[d] * (1.0 - t[d] ** 2)
                  if d == m else c[d] for d in range(3)]
            N[a] = 9.0 * f[0] * f[1] * f[2] / 64.0
            G[a, 0] = 9.0 * df[0] * f[1] * f[2] / 64.0
            G[a, 1] = 9.0 * f[0] * df[1] * f[2] / 64.0
            G[a, 2] = 9.0 * f[0] * f[1] * df[2] / 64.0
    return N, G


def serendipity_shapes(xi, eta, zeta, order=2):
    """Values [(p+1)^3] and local gradients [(p+1)^3, 3] of the serendipity
    shape functions of degree p = order (2: 20 nodes, 3: 32 nodes) in the
    Lagrange layout of the same degree (zero at the nodes the element does
    not have)."""
    if order == 2:
        return _serendipity2(xi, eta, zeta)
    if order == 3:
        return _serendipity3(xi, eta, zeta)
    raise ValueError("serendipity elements here have degree 2 or 3")


def strain_displacement(order, xi, eta, zeta, half=(0.5, 0.5, 0.5), family="lagrange"):
    """B (6 x 3*n_e) at one local point of an element of half-sizes
    (l, h, w); family "serendipity" (order 2 or 3) keeps the Lagrange layout
    of its degree."""
    p1 = order + 1
    nen = p1 ** 3
    B = np.zeros((6, 3 * nen))
    if family == "serendipity":
        _, G = serendipity_shapes(xi, eta, zeta, order)
        G = G / np.asarray(half)
    else:
        _, val, der = lagrange_1d(order)
        vx, vy, vz = val(xi), val(eta), val(zeta)
        dx, dy, dz = der(xi) / half[0], der(eta) / half[1], der(zeta) / half[2]
    for az in range(p1):
        for ay in range(p1):
            for ax in range(p1):
                a = ax + p1 * (ay + p1 * az)
                if family == "serendipity":
                    gx, gy, gz = G[a]
                else:
                    gx = dx[ax] * vy[ay] * vz[az]
                    gy = vx[ax] * dy[ay] * vz[az]
                    gz = vx[ax] * vy[ay] * dz[az]
                u, v, w = 3 * a, 3 * a + 1, 3 * a + 2
                B[0, u] = gx
                B[1, v] = gy
                B[2, w] = gz
                B[3, u], B[3, v] = gy, gx
                B[4, v], B[4, w] = gz, gy
                B[5, w], B[5, u] = gx, gz
    return B


def sub_element_matrices(order, nsub, nu=0.3, E=1.0, half=(0.5, 0.5, 0.5), family="lagrange"):
    """The n^3 matrices K^(e_i) of one displacement element (Sec. 3.3), as an
    array [n^3, 3n_e, 3n_e]; sub-element i = sx + n*(sy + n*sz)."""
    D = elasticity_matrix(E, nu)
    gp, gw = np.polynomial.legendre.leggauss(order + 1)
    jac = half[0] * half[1] * half[2]
    nen = (order + 1) ** 3
    out = np.zeros((nsub ** 3, 3 * nen, 3 * nen))
    edges = np.linspace(-1.0, 1.0, nsub + 1)
    for sz in range(nsub):
        for sy in range(nsub):
            for sx in range(nsub):
                K = np.zeros((3 * nen, 3 * nen))
                lo = (edges[sx], edges[sy], edges[sz])
                hi = (edges[sx + 1], edges[sy + 1], edges[sz + 1])
                mid = [(a + b) / 2 for a, b in zip(lo, hi)]
                rad = [(b - a) / 2 for a, b in zip(lo, hi)]
                for qz, wz in zip(gp, gw):
                    for qy, wy in zip(gp, gw):
                        for qx, wx in zip(gp, gw):
                            B = strain_displacement(
                                order, mid[0] + rad[0] * qx, mid[1] + rad[1] * qy,
                                mid[2] + rad[2] * qz, half, family)
                            wgt = wx * wy * wz * rad[0] * rad[1] * rad[2] * jac
                            K += wgt * (B.T @ D @ B)
                out[sx + nsub * (sy + nsub * sz)] = K
    return out


def element_matrix(order, nu=0.3, E=1.0, family="lagrange"):
    """Single-resolution element stiffness, integral over the whole element."""
    return sub_element_matrices(order, 1, nu, E, family=family)[0]


def serendipity_dof_mask(nel, order=2):
    """DOF mask (3 per node) of the Lagrange lattice of degree `order` of a
    mesh, marking the face-interior and body-interior nodes (two or three
    lattice indices strictly inside an element's edge), which no
    serendipity element uses."""
    nelx, nely, nelz = nel
    i = (np.arange(order * nelx + 1) % order != 0).astype(int)
    j = (np.arange(order * nely + 1) % order != 0).astype(int)
    k = (np.arange(order * nelz + 1) % order != 0).astype(int)
    inner = k[:, None, None] + j[None, :, None] + i[None, None, :]
    return np.repeat((inner >= 2).reshape(-1), 3).astype(np.uint8)


def local_node_coords(order):
    """Physical coordinates (unit element, origin at the corner) of the local
    nodes, shape [n_e, 3]."""
    p1 = order + 1
    t = np.linspace(0.0, 1.0, p1)
    out = []
    for az in range(p1):
        for ay in range(p1):
            for ax in range(p1):
                out.append((t[ax], t[ay], t[az]))
    return np.array(out)


def rigid_body_modes(coords):
    """Six rigid-body displacement fields (3 translations, 3 infinitesimal
    rotations) sampled at the given node coordinates, shape [6, 3*n]."""
    n = coords.shape[0]
    R = np.zeros((6, 3 * n))
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    for c in range(3):
        R[c, c::3] = 1.0
    # rotation about z: (-y, x, 0); about x: (0, -z, y); about y: (z, 0, -x)
    R[3, 0::3], R[3, 1::3] = -y, x
    R[4, 1::3], R[4, 2::3] = -z, y
    R[5, 0::3], R[5, 2::3] = z, -x
    return R
