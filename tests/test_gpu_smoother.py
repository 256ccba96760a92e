"""GPU parity of the multicolour Gauss-Seidel smoother on the quadratic
finest level (Sec. 7.5 smooths quadratic elements by SSOR): the V-cycle
against the oracle's Algorithm 1 with the same sweeps (forward before,
backward after the coarse correction), and MGCG solves against the oracle's
direct solve, with Lagrange and serendipity elements, FP64 and mixed
precision, one to four load cases."""

import numpy as np
import pytest

from helpers import Case, need_gpu, rel

pytestmark = pytest.mark.gpu

GS = "gauss-seidel"

VCYCLE_CASES = [
    ("cantilever", (4, 2, 2), 2, 2, 2, "fp64"),
    ("torsion", (6, 4, 4), 1, 3, 3, "fp64"),
    ("mbb", (5, 3, 3), 1, 2, 4, "fp64"),     # odd element counts: boundary colours
    ("cantilever", (4, 2, 2), 4, 2, 1, "fp64"),
    ("cantilever", (6, 4, 4), 2, 3, 2, "mixed"),
]


@pytest.mark.parametrize("kind,nel,nsub,nlev,nrhs,prec", VCYCLE_CASES)
def test_gs_vcycle_matches_oracle(kind, nel, nsub, nlev, nrhs, prec):
    need_gpu()
    from oracle import multigrid
    c = Case(kind, nel, 2, nsub, nlev, nrhs, seed=61, precision=prec)
    p = c.problem(smoother=GS)
    p.set_densities(c.rho)
    r = np.random.default_rng(62).standard_normal((nrhs, p.ndof))
    r[:, c.mask.astype(bool)] = 0.0
    z = p.precondition(r)
    tol = 1e-9 if prec == "fp64" else 1e-4
    for l in range(nrhs):
        assert rel(z[l], multigrid.vcycle(c.H, r[l], omega=c.omega, smoother="gs")) <= tol, l
    p.close()


SOLVE_CASES = [
    ("cantilever", (8, 4, 4), 1, 3, 1, "fp64"),
    ("cantilever", (6, 2, 2), 4, 2, 2, "fp64"),
    ("torsion", (4, 2, 2), 2, 2, 4, "mixed"),
    ("mbb", (8, 4, 4), 2, 3, 3, "mixed"),
]


@pytest.mark.parametrize("kind,nel,nsub,nlev,nrhs,prec", SOLVE_CASES)
def test_gs_solve_matches_direct(kind, nel, nsub, nlev, nrhs, prec):
    need_gpu()
    c = Case(kind, nel, 2, nsub, nlev, nrhs, seed=63, precision=prec)
    p = c.problem(smoother=GS)
    p.set_densities(c.rho)
    info = p.solve(rtol=1e-10, maxit=3000, warm_start=False)
    assert info["status"] == 0
    u = p.displacement()
    cc, dc = p.compliance_sensitivity()
    p.close()
    ud = c.direct()
    for l in range(nrhs):
        assert rel(u[l], ud[l]) <= 1e-8, l
    cref = c.compliance(ud)
    assert np.all(np.abs(cc[:nrhs] - cref) <= 1e-9 * np.abs(cref))
    assert rel(dc, c.sensitivity(ud)) <= 1e-8


def test_gs_takes_fewer_iterations_than_jacobi():
    """Sec. 7.5: for quadratic elements the Gauss-Seidel smoother beats the
    (capped) Jacobi sweep; on a rough n = 4 field by a wide margin."""
    need_gpu()
    c = Case("cantilever", (8, 4, 4), 2, 4, 3, 1, seed=64)
    its = {}
    for sm in ("jacobi", GS):
        p = c.problem(smoother=sm)
        p.set_densities(c.rho)
        its[sm] = p.solve(rtol=1e-10, maxit=3000, warm_start=False)["iters"][0]
        p.close()
    assert its[GS] * 2 <= its["jacobi"], its


@pytest.mark.parametrize("nel,n,nrhs,prec", [((6, 4, 2), 2, 1, "fp64"), ((4, 2, 2), 2, 3, "mixed")])
def test_gs_serendipity_solve_matches_oracle(nel, n, nrhs, prec):
    need_gpu()
    import workloads as W
    from oracle import fem, solve
    from paper_2311_05595_amd import api
    mask, f = W.make_problem("cantilever", *nel, 2, nrhs)
    rho = np.random.default_rng(65).uniform(0.1, 1.0, (n * nel[2], n * nel[1], n * nel[0]))
    p = api.Problem(nel, mask, f, order=2, nsub=n, nlevels=2, precision=prec,
                    family="serendipity", smoother=GS)
    p.set_densities(rho.reshape(-1))
    info = p.solve(rtol=1e-11, maxit=3000, warm_start=False)
    assert info["status"] == 0
    u = p.displacement()
    c, _ = p.compliance_sensitivity(want_dc=False)
    p.close()
    ms = np.maximum(mask, fem.serendipity_dof_mask(nel))
    Ks = fem.sub_element_matrices(2, n, family="serendipity")
    _, u_o, c_o, _ = solve.solve_problem(rho, ms, f, nel, 2, n, Ks, E0=1.0, Emin=1e-9, penal=3.0)
    u_o = np.asarray(u_o).reshape(nrhs, -1)
    for lc in range(nrhs):
        assert np.all(u[lc][ms.astype(bool)] == 0.0)
        assert np.linalg.norm(u[lc] - u_o[lc]) <= 1e-8 * np.linalg.norm(u_o[lc]), lc
        assert abs(c[lc] - c_o[lc]) <= 1e-9 * abs(c_o[lc]), lc
