"""Choice of the variables that are fixed before the degree of the elements is
raised (Sec. 6.1), as plain definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* A displacement element is void when every density inside it is
  <= rho_l and every design-gradient component inside it is >= -eps, and
  solid when every density is >= rho_u and every gradient component
  <= eps (rho_l = 1e-6, rho_u = 0.9, eps = 1e-6 in the paper).
* Only elements surrounded by elements of their own kind are fixed.
  Reading: the neighbours are the elements that share at least one node with
  it (up to 26), those outside the domain do not count.
* The design variables inside fixed (void or solid) elements are fixed.
* The nodes whose displacements are suppressed are the nodes of the
  displacement lattice (of the raised degree) all of whose elements are
  fixed void elements.  Reading: "internal nodes of the void elements" taken
  as nodes touched by no other element, so that no element outside the
  fixed void region loses a node; the suppressed DOFs join the supports.

Lattices are (z, y, x) arrays, x fastest: the densities have n cells per
element and axis, the design variables d, the nodes order * nel + 1.

Pins (tests/test_oracle_fixing.py): hand-counted cases (a void block, a
solid block, the domain boundary, a gradient that vetoes), the surrounded
rule against scipy.ndimage's binary erosion with a full 3x3x3 element, and
the physical claim of Sec. 6.1: with E_min = 1e-9 the compliance changes by
a negligible amount when the suppressed DOFs are fixed.
"""

import numpy as np

MIXED, VOID, SOLID = 0, 1, 2


def classify(rho, grad, nel, n, d, rho_l=1e-6, rho_u=0.9, eps=1e-6):
    """Kind of every element (MIXED, VOID, SOLID), shape (nelz, nely, nelx)."""
    nelx, nely, nelz = nel
    rho = np.asarray(rho, dtype=np.float64).reshape(n * nelz, n * nely, n * nelx)
    grad = np.asarray(grad, dtype=np.float64).reshape(d * nelz, d * nely, d * nelx)
    kind = np.zeros((nelz, nely, nelx), dtype=np.uint8)
    for ez in range(nelz):
        for ey in range(nely):
            for ex in range(nelx):
                r = rho[n * ez:n * ez + n, n * ey:n * ey + n, n * ex:n * ex + n]
                g = grad[d * ez:d * ez + d, d * ey:d * ey + d, d * ex:d * ex + d]
                if np.all(r <= rho_l) and np.all(g >= -eps):
                    kind[ez, ey, ex] = VOID
                elif np.all(r >= rho_u) and np.all(g <= eps):
                    kind[ez, ey, ex] = SOLID
    return kind


def surrounded(kind):
    """Fixed kind per element: VOID or SOLID when the element and every
    neighbour inside the domain share that kind, MIXED otherwise."""
    nz, ny, nx = kind.shape
    out = np.zeros_like(kind)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                k = kind[z, y, x]
                if k == MIXED:
                    continue
                same = True
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            zz, yy, xx = z + dz, y + dy, x + dx
                            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                                same = same and kind[zz, yy, xx] == k
                out[z, y, x] = k if same else MIXED
    return out


def fixed_design(fixed_kind, d):
    """1 for the design variables inside fixed elements (design lattice)."""
    f = (fixed_kind != MIXED).astype(np.uint8)
    return np.repeat(np.repeat(np.repeat(f, d, axis=0), d, axis=1), d, axis=2)


def suppressed_nodes(fixed_kind, order):
    """1 for the nodes (lattice of the given order) whose elements are all
    fixed void elements."""
    nelz, nely, nelx = fixed_kind.shape
    dims = (order * nelz + 1, order * nely + 1, order * nelx + 1)
    out = np.zeros(dims, dtype=np.uint8)

    def elems(i, nel):
        # elements along one axis that contain node index i of that axis
        if i % order:
            return [i // order]
        return [e for e in (i // order - 1, i // order) if 0 <= e < nel]

    for k in range(dims[0]):
        for j in range(dims[1]):
            for i in range(dims[2]):
                ok = True
                for ez in elems(k, nelz):
                    for ey in elems(j, nely):
                        for ex in elems(i, nelx):
                            ok = ok and fixed_kind[ez, ey, ex] == VOID
                out[k, j, i] = 1 if ok else 0
    return out


def dof_mask(support_mask, nodes):
    """The supports' DOF mask (3 per node) with the suppressed nodes' DOFs."""
    m = np.array(support_mask, dtype=np.uint8).copy()
    m[np.repeat(nodes.reshape(-1) != 0, 3)] = 1
    return m


__all__ = ["MIXED", "VOID", "SOLID", "classify", "surrounded", "fixed_design",
           "suppressed_nodes", "dof_mask"]
