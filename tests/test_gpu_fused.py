"""The fused small-problem solve (one workgroup per load case runs the whole
PCG solve with its V-cycle, Sec. 2.3 and Algorithm 1) and the batched
multi-problem launch: against the oracle's direct solve (u to 1e-8, c to
1e-9 at a relative residual of 1e-12), against the eagerly launched solve of
the same problem (u to 1e-9), with warm starts, and several problems of
different meshes and load counts in one launch."""

import numpy as np
import pytest

from helpers import MAT, Case, need_gpu, rel

pytestmark = pytest.mark.gpu

CASES = [
    # kind, nel, nlevels, nrhs
    ("cantilever", (8, 4, 4), 3, 1),
    ("mbb", (12, 8, 4), 3, 2),
    ("torsion", (10, 6, 6), 2, 3),
    ("cantilever", (24, 12, 12), 3, 4),   # 4225 nodes: the small benchmark mesh
    # 5577 nodes; its second level (833 nodes) fills 60 % of the LDS that the
    # stencil levels' pair sums may take
    ("cantilever", (32, 12, 12), 3, 2),
]


def _id(c):
    return f"{c[0]}-{'x'.join(map(str, c[1]))}-L{c[2]}-r{c[3]}"


@pytest.mark.parametrize("kind,nel,nlevels,nrhs", CASES, ids=[_id(c) for c in CASES])
def test_fused_solve_matches_oracle_and_eager(kind, nel, nlevels, nrhs):
    need_gpu()
    # uniform densities in [0.05, 1] (the small benchmark's field): with
    # void regions some load cases stall above 1e-12
    c = Case(kind, nel, 1, 1, nlevels, nrhs, seed=41, field="uniform")
    out = {}
    for mode in ("eager", "fused"):
        p = c.problem()
        p.set_densities(c.rho.reshape(-1))
        p.set_launch_mode(mode)
        info = p.solve(rtol=1e-12, maxit=2000, warm_start=False, allow_notconv=True)
        assert max(info["rel_res"][:nrhs]) <= 2e-12, (mode, info)
        cc, dc = p.compliance_sensitivity()
        out[mode] = (p.displacement(), cc, dc, info["iters"][:nrhs])
        p.close()
    u, cc, dc, its = out["fused"]
    ue, _, _, its_e = out["eager"]
    ud = c.direct()
    co = c.compliance(ud)
    for lc in range(nrhs):
        assert rel(u[lc], ud[lc]) <= 1e-8, lc
        assert abs(cc[lc] - co[lc]) <= 1e-9 * abs(co[lc]), lc
        assert rel(u[lc], ue[lc]) <= 1e-9, lc
        # the same iteration in another summation order
        assert abs(its[lc] - its_e[lc]) <= 2, (its, its_e)
    assert rel(dc, out["eager"][2]) <= 1e-9


def test_fused_warm_start_and_notconv():
    need_gpu()
    c = Case("cantilever", (16, 8, 8), 1, 1, 3, 2, seed=43, field="uniform")
    p = c.problem()
    p.set_densities(c.rho.reshape(-1))
    p.set_launch_mode("fused")
    cold = p.solve(rtol=1e-10, maxit=2000, warm_start=False)
    rho2 = np.clip(c.rho + 0.02 * np.random.default_rng(3).uniform(-1, 1, c.rho.shape), 1e-3, 1.0)
    p.set_densities(rho2.reshape(-1))
    warm = p.solve(rtol=1e-10, maxit=2000, warm_start=True)
    assert warm["status"] == 0 and max(warm["rel_res"][:2]) <= 1e-10
    from oracle import assemble, solve
    K = assemble.stiffness(rho2, c.nel, 1, 1, c.Ks, **MAT)
    ud = solve.solve_direct(K, c.mask, c.f)
    u = p.displacement()
    for lc in range(2):
        assert rel(u[lc], ud[lc]) <= 1e-8
    assert sum(warm["iters"][:2]) < sum(cold["iters"][:2])
    # too few iterations: the solve stops at maxit with ENOTCONV
    p.set_densities(c.rho.reshape(-1))
    info = p.solve(rtol=1e-12, maxit=3, warm_start=False, allow_notconv=True)
    assert info["status"] != 0 and info["iters"][:2] == [3, 3]
    p.close()


def test_batched_multi_problem_launch():
    """Six problems (three meshes, 1-4 load cases, two of them warm-started)
    in one launch give what each gives solved alone."""
    need_gpu()
    from paper_2311_05595_amd import api
    specs = [("cantilever", (8, 4, 4), 3, 1), ("mbb", (12, 8, 4), 3, 2),
             ("torsion", (10, 6, 6), 2, 3), ("cantilever", (24, 12, 12), 3, 4),
             ("mbb", (8, 8, 4), 3, 1), ("cantilever", (6, 2, 2), 2, 2)]
    cases = [Case(k, n, 1, 1, l, r, seed=50 + i, field="uniform")
             for i, (k, n, l, r) in enumerate(specs)]
    alone, batch = [], []
    for c in cases:
        p = c.problem()
        p.set_densities(c.rho.reshape(-1))
        p.solve(rtol=1e-11, maxit=2000, warm_start=False)
        alone.append(p.displacement())
        p.close()
        q = c.problem()
        q.set_densities(c.rho.reshape(-1))
        batch.append(q)
    infos = api.solve_batch(batch, rtol=1e-11, maxit=2000, warm_start=False)
    for c, q, info, ua in zip(cases, batch, infos, alone):
        assert info["status"] == 0
        assert max(info["rel_res"][:c.nrhs]) <= 1e-11
        u = q.displacement()
        for lc in range(c.nrhs):
            assert rel(u[lc], ua[lc]) <= 1e-9
    # a second batch, warm-started from the first solutions, on new densities
    for c, q in zip(cases, batch):
        rho2 = np.clip(c.rho * 1.01, 0.0, 1.0)
        q.set_densities(rho2.reshape(-1))
    infos2 = api.solve_batch(batch, rtol=1e-11, maxit=2000, warm_start=True)
    assert all(i["status"] == 0 for i in infos2)
    for q in batch:
        q.close()


@pytest.mark.parametrize("pre,post", [(2, 2), (3, 1)])
def test_fused_smoothing_counts(pre, post):
    """More than one smoothing sweep per level (the loops of the fused
    V-cycle): the preconditioner matches Algorithm 1 through the solve's
    iterates, so the fused solve agrees with the eager one and the oracle."""
    need_gpu()
    c = Case("mbb", (16, 8, 8), 1, 1, 4, 2, seed=47, field="uniform")
    out = {}
    for mode in ("eager", "fused"):
        p = c.problem(pre=pre, post=post)
        p.set_densities(c.rho.reshape(-1))
        p.set_launch_mode(mode)
        info = p.solve(rtol=1e-12, maxit=2000, warm_start=False, allow_notconv=True)
        assert max(info["rel_res"][:2]) <= 2e-12, (mode, info)
        out[mode] = (p.displacement(), info["iters"][:2])
        p.close()
    ud = c.direct()
    for lc in range(2):
        assert rel(out["fused"][0][lc], ud[lc]) <= 1e-8
        assert abs(out["fused"][1][lc] - out["eager"][1][lc]) <= 2
