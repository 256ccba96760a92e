"""Contexts (a device and a shared HBM budget) and FP32 density input on the
GPU: a problem's first allocation is charged to its context, refused with
MGCG_EBUDGET when the budget cannot hold it, refunded when it is destroyed;
FP32 densities (host or device) give the solve of their FP64 values."""

import numpy as np
import pytest

from helpers import need_gpu

pytestmark = pytest.mark.gpu


def test_context_budget_charges_and_refunds():
    need_gpu()
    import workloads as W
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError, MGCG_EBUDGET
    nel = (8, 4, 4)
    mask, f = W.make_problem("cantilever", *nel, 1, 1)
    rho = np.full(nel[0] * nel[1] * nel[2], 0.5)
    need = api.device_bytes(nel=nel, nlevels=2)
    ctx = api.Context(0, budget=need + need // 2)  # room for one problem, not two
    p1 = api.Problem(nel, mask, f, nlevels=2, ctx=ctx)
    p2 = api.Problem(nel, mask, f, nlevels=2, ctx=ctx)
    p1.set_densities(rho)
    assert ctx.usage() == (need, need + need // 2, 2)
    with pytest.raises(MGCGError) as ei:
        p2.set_densities(rho)
    assert ei.value.code == MGCG_EBUDGET
    assert ctx.usage()[0] == need
    p1.close()
    assert ctx.usage() == (0, need + need // 2, 1)
    p2.set_densities(rho)
    assert p2.solve(rtol=1e-8, warm_start=False)["status"] == 0
    assert ctx.usage()[0] == need
    p2.close()
    ctx.close()


def test_fp32_densities_solve_their_fp64_values():
    need_gpu()
    import torch
    import workloads as W
    from paper_2311_05595_amd import api
    nel = (8, 4, 4)
    mask, f = W.make_problem("cantilever", *nel, 1, 2)
    rho32 = W.gaussian_random_field((4, 4, 8), 5, corr=3.0).astype(np.float32).ravel()
    out = []
    for src in (rho32.astype(np.float64), rho32, torch.tensor(rho32, device="cuda")):
        p = api.Problem(nel, mask, f, nlevels=2)
        p.set_densities(src)
        p.solve(rtol=1e-10, warm_start=False)
        out.append((p.displacement(), p.compliance_sensitivity()))
        p.close()
    for u, (c, dc) in out[1:]:
        assert np.array_equal(u, out[0][0])
        assert np.array_equal(c, out[0][1][0])
        assert np.array_equal(dc, out[0][1][1])
