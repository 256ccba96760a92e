"""GPU parity of the design-variable projection / density filter (Sec. 3.2
eq. (5) with the weights of Sec. 2.2 eq. (4)) and its transpose (the chain
rule of Sec. 3.4) against the oracle, through the C ABI.

Two kernel paths are covered: tiled gathers over precomputed phase stencils
(n a multiple of d, stencils within 4 design cells) and plain per-cell
searches (the other cases: d not dividing n, very large radii).

Tolerances: every output is a sum of at most a few thousand positive-weight
FP64 products, evaluated in a different order (and with the weight as a
product of three per-axis factors instead of one exponential), so outputs
agree to a few ulps of their magnitude: 1e-13 relative to the largest
output."""

import numpy as np
import pytest

from oracle import projection as P
from tests.helpers import need_gpu

pytestmark = pytest.mark.gpu

CASES = [
    # nel, n (density cells per element), d (design cells), rmin
    ((6, 4, 3), 4, 2, 0.6),      # multiresolution, paper's small radius
    ((5, 3, 2), 1, 1, 1.5),      # plain density filter
    ((4, 2, 2), 2, 1, 0.8),
    ((3, 3, 2), 4, 4, 1.3),      # filter on the density lattice
    ((4, 3, 2), 2, 2, 2.0),
    ((7, 2, 3), 3, 1, 0.9),      # n not a power of two, ragged lattice
    ((2, 2, 2), 2, 4, 0.7),      # more design cells than density cells
    ((3, 1, 1), 1, 1, 1.0),      # neighbours exactly on the ball's boundary
    ((1, 1, 1), 4, 2, 0.25),     # one element
    ((3, 2, 2), 2, 1, 10.0),     # every ball holds the whole domain
    ((9, 5, 3), 4, 2, 1.5),      # several tiles with ragged edges, the benchmark's stencil
    ((17, 9, 5), 2, 2, 1.0),
]


def _proj(nel, n, d, rmin):
    from paper_2311_05595_amd import api
    return api.Projection(nel, n, d, rmin)


@pytest.mark.parametrize("nel,n,d,rmin", CASES)
def test_forward_and_transpose_match_oracle(nel, n, d, rmin):
    need_gpu()
    import torch
    rng = np.random.default_rng(hash((nel, n, d)) % 2 ** 32)
    Wm = P.projection_matrix(nel, n, d, rmin)
    x = rng.random(Wm.shape[1])
    g = rng.standard_normal(Wm.shape[0])
    pr = _proj(nel, n, d, rmin)
    rho = pr.apply(x)
    gx = pr.apply_transpose(g)
    rho_o, gx_o = Wm @ x, Wm.T @ g
    assert np.abs(rho - rho_o).max() <= 1e-13 * np.abs(rho_o).max()
    assert np.abs(gx - gx_o).max() <= 1e-13 * np.abs(gx_o).max()
    # the device-memory path returns the same bits
    xd = torch.tensor(x, device="cuda")
    gd = torch.tensor(g, device="cuda")
    rd = pr.apply(xd)
    gxd = pr.apply_transpose(gd)
    torch.cuda.synchronize()
    assert np.array_equal(rd.cpu().numpy(), rho)
    assert np.array_equal(gxd.cpu().numpy(), gx)
    pr.close()


def test_full_size_sampled_and_properties():
    """The 64x32x32 mesh with 4^3 density cells and 2^3 design cells per
    element (4.2M densities, 524k design variables), rmin = 1.5: sampled
    entries against the oracle's single-entry evaluation, W 1 = 1 everywhere
    and the adjoint identity <W x, g> = <x, W^T g>."""
    need_gpu()
    import torch
    nel, n, d, rmin = (64, 32, 32), 4, 2, 1.5
    pr = _proj(nel, n, d, rmin)
    rng = np.random.default_rng(7)
    Sr, Sx = P.lattice_shape(nel, n), P.lattice_shape(nel, d)
    x = rng.random(pr.nx)
    g = rng.standard_normal(pr.nrho)
    xd = torch.tensor(x, device="cuda")
    gd = torch.tensor(g, device="cuda")
    rho = pr.apply(xd).cpu().numpy()
    gx = pr.apply_transpose(gd).cpu().numpy()
    # corners, faces and random interior cells
    picks = [0, pr.nrho - 1, Sr[2] - 1, Sr[2] * Sr[1] - 1] + list(rng.choice(pr.nrho, 200))
    for flat in picks:
        i3 = (flat % Sr[2], (flat // Sr[2]) % Sr[1], flat // (Sr[2] * Sr[1]))
        ref = P.project_at(x, i3, nel, n, d, rmin)
        assert abs(rho[flat] - ref) <= 1e-13, (i3, rho[flat], ref)
    gscale = np.abs(gx).max()
    for flat in [0, pr.nx - 1] + list(rng.choice(pr.nx, 24)):
        k3 = (flat % Sx[2], (flat // Sx[2]) % Sx[1], flat // (Sx[2] * Sx[1]))
        ref = P.project_transpose_at(g, k3, nel, n, d, rmin)
        assert abs(gx[flat] - ref) <= 1e-13 * gscale, (k3, gx[flat], ref)
    ones = pr.apply(torch.ones(pr.nx, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.abs(ones - 1.0).max() <= 1e-14
    lhs, rhs = float(rho @ g), float(x @ gx)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(rho) @ np.abs(g))
    pr.close()


def test_autograd_chain_rule_matches_oracle():
    """x -> rho = W x -> compliance: x.grad = W^T dc (Sec. 3.4), against the
    oracle's direct solve and transpose."""
    need_gpu()
    import torch
    from oracle import fem, solve
    import workloads as W
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd.autograd import compliance, project
    nel, n, d, rmin = (4, 2, 2), 2, 1, 0.9
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    prob = api.Problem(nel, mask, f, nsub=n, nlevels=2)
    pr = _proj(nel, n, d, rmin)
    rng = np.random.default_rng(3)
    x0 = 0.3 + 0.6 * rng.random(pr.nx)
    x = torch.tensor(x0, device="cuda", requires_grad=True)
    c = compliance(project(x, pr), prob, rtol=1e-12)
    c.backward()
    gx = x.grad.cpu().numpy()
    Wm = P.projection_matrix(nel, n, d, rmin)
    rho_o = (Wm @ x0).reshape(P.lattice_shape(nel, n))
    Ks = fem.sub_element_matrices(1, n)
    _, _, c_o, dc_o = solve.solve_problem(rho_o, mask, f, nel, 1, n, Ks, E0=1.0, Emin=1e-9,
                                          penal=3.0)
    gx_o = Wm.T @ dc_o
    assert abs(float(c.detach()) - c_o.sum()) <= 1e-9 * c_o.sum()
    assert np.abs(gx - gx_o).max() <= 1e-8 * np.abs(gx_o).max()
    pr.close()
    prob.close()
