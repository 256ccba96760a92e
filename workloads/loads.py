"""Supports and nodal loads of the test structures (cantilever, MBB beam,
torsion box), as input data for both the oracle and the HIP library.

Every builder returns ``(mask, f)``:

* ``mask``: ``uint8[ndof]``, 1 where the DOF is fixed (supported), else 0;
* ``f``: ``float64[nrhs, ndof]`` nodal loads, zero on fixed DOFs.

Distributed loads use consistent nodal weights of the element's shape
functions on a uniform lattice: for linear elements the trapezoid weights
(1/2 at the ends of each element edge), for quadratic elements Simpson's
weights (1/6, 4/6, 1/6 per element), for cubic ones Simpson's 3/8 weights
(1/8, 3/8, 3/8, 1/8 per element).  Point loads are shared equally by the
nearest lattice nodes when the target point is not a node.
"""

import numpy as np


def node_dims(nelx, nely, nelz, order=1):
    return (order * nelx + 1, order * nely + 1, order * nelz + 1)


def _line_weights(nel, order):
    """Consistent weights of a unit load per unit length on a line of `nel`
    unit elements of the given order (sum = nel)."""
    n = order * nel + 1
    w = np.zeros(n)
    if order == 1:
        per = np.array([0.5, 0.5])
    elif order == 2:
        per = np.array([1.0, 4.0, 1.0]) / 6.0
    elif order == 3:
        per = np.array([1.0, 3.0, 3.0, 1.0]) / 8.0
    else:
        raise ValueError("order must be 1, 2 or 3")
    for e in range(nel):
        w[order * e: order * e + order + 1] += per
    return w


def _node(i, j, k, dims):
    nx, ny, _ = dims
    return i + nx * (j + ny * k)


def _point(f, dims, x, y, z, comp, value):
    """Add a point force at lattice coordinates (x, y, z) (possibly
    fractional), shared by the surrounding lattice nodes."""
    xs = [int(np.floor(x)), int(np.ceil(x))] if x != int(x) else [int(x)]
    ys = [int(np.floor(y)), int(np.ceil(y))] if y != int(y) else [int(y)]
    zs = [int(np.floor(z)), int(np.ceil(z))] if z != int(z) else [int(z)]
    share = value / (len(xs) * len(ys) * len(zs))
    for i in xs:
        for j in ys:
            for k in zs:
                f[3 * _node(i, j, k, dims) + comp] += share


def _face_fix(mask, dims, axis, index):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sel = [i, j, k][axis] == index
    nodes = (i + nx * (j + ny * k))[sel]
    for c in range(3):
        mask[3 * nodes + c] = 1


def _load_tip(dims, nel, order):
    """Unit -y load spread over the bottom edge {x = max, y = 0}."""
    nx, ny, nz = dims
    f = np.zeros(3 * nx * ny * nz)
    w = _line_weights(nel[2], order)
    w = w / w.sum()
    for k in range(nz):
        f[3 * _node(nx - 1, 0, k, dims) + 1] -= w[k]
    return f


def _load_lateral(dims, nel, order):
    """Unit +z load spread over the mid-height edge {x = max, z = max}."""
    nx, ny, nz = dims
    f = np.zeros(3 * nx * ny * nz)
    w = _line_weights(nel[1], order)
    w = w / w.sum()
    for j in range(ny):
        f[3 * _node(nx - 1, j, nz - 1, dims) + 2] += w[j]
    return f


def pressure_load(dims, nel, order, value=1.0):
    """Uniform pressure `value` per unit area, acting in -y on the top face."""
    nx, ny, nz = dims
    f = np.zeros(3 * nx * ny * nz)
    wx = _line_weights(nel[0], order)
    wz = _line_weights(nel[2], order)
    for k in range(nz):
        for i in range(nx):
            f[3 * _node(i, ny - 1, k, dims) + 1] -= value * wx[i] * wz[k]
    return f


def _load_torque(dims, nel, order):
    """Tangential tractions on the face x = max forming a unit torque about
    the x-axis through the face centroid."""
    nx, ny, nz = dims
    f = np.zeros(3 * nx * ny * nz)
    wy = _line_weights(nel[1], order)
    wz = _line_weights(nel[2], order)
    yc, zc = nel[1] / 2.0, nel[2] / 2.0
    jj = 0.0
    for k in range(nz):
        for j in range(ny):
            y, z = j / order - yc, k / order - zc
            jj += wy[j] * wz[k] * (y * y + z * z)
    for k in range(nz):
        for j in range(ny):
            y, z = j / order - yc, k / order - zc
            w = wy[j] * wz[k] / jj
            n = _node(nx - 1, j, k, dims)
            f[3 * n + 1] -= w * z
            f[3 * n + 2] += w * y
    return f


def _load_top_point(dims, frac_x):
    nx, ny, nz = dims
    f = np.zeros(3 * nx * ny * nz)
    _point(f, dims, frac_x * (nx - 1), ny - 1, 0.5 * (nz - 1), 1, -1.0)
    return f


def _finish(mask, loads):
    f = np.stack(loads).astype(np.float64)
    f[:, mask.astype(bool)] = 0.0
    return mask, f


_CANTILEVER_LOADS = ("tip", "pressure", "torque", "lateral")
_MBB_LOADS = ("center", "pressure", "quarter", "lateral")
_TORSION_LOADS = ("torque", "tip", "pressure", "lateral")


def _build_loads(names, dims, nel, order):
    out = []
    for name in names:
        if name == "tip":
            out.append(_load_tip(dims, nel, order))
        elif name == "pressure":
            out.append(pressure_load(dims, nel, order))
        elif name == "torque":
            out.append(_load_torque(dims, nel, order))
        elif name == "lateral":
            out.append(_load_lateral(dims, nel, order))
        elif name == "center":
            out.append(_load_top_point(dims, 0.5))
        elif name == "quarter":
            out.append(_load_top_point(dims, 0.25))
        else:
            raise ValueError(name)
    return out


def cantilever_bcs(nelx, nely, nelz, order=1, loads=("tip",)):
    """x = 0 face clamped; loads at the free end x = nelx."""
    dims = node_dims(nelx, nely, nelz, order)
    mask = np.zeros(3 * dims[0] * dims[1] * dims[2], dtype=np.uint8)
    _face_fix(mask, dims, 0, 0)
    return _finish(mask, _build_loads(loads, dims, (nelx, nely, nelz), order))


def torsion_bcs(nelx, nely, nelz, order=1, loads=("torque",)):
    """Torsion box: x = 0 face clamped, unit torque on the face x = nelx."""
    return cantilever_bcs(nelx, nely, nelz, order, loads)


def mbb_bcs(nelx, nely, nelz, order=1, loads=("center",)):
    """MBB beam: every DOF fixed at the nodes of the bottom face of each of the
    four bottom-corner elements; unit -y load at the top-face centre."""
    dims = node_dims(nelx, nely, nelz, order)
    nx, ny, nz = dims
    mask = np.zeros(3 * nx * ny * nz, dtype=np.uint8)
    xs = list(range(0, order + 1)) + list(range(nx - 1 - order, nx))
    zs = list(range(0, order + 1)) + list(range(nz - 1 - order, nz))
    for k in zs:
        for i in xs:
            n = _node(i, 0, k, dims)
            mask[3 * n: 3 * n + 3] = 1
    return _finish(mask, _build_loads(loads, dims, (nelx, nely, nelz), order))


def make_problem(kind, nelx, nely, nelz, order=1, nrhs=1):
    """Supports and the first `nrhs` load cases of a named structure."""
    if kind == "cantilever":
        return cantilever_bcs(nelx, nely, nelz, order, _CANTILEVER_LOADS[:nrhs])
    if kind == "mbb":
        return mbb_bcs(nelx, nely, nelz, order, _MBB_LOADS[:nrhs])
    if kind == "torsion":
        return torsion_bcs(nelx, nely, nelz, order, _TORSION_LOADS[:nrhs])
    raise ValueError(kind)
