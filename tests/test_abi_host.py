"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, validates descriptions, sizes problems and
plans admissions."""

import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2311_05595_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libmgcg.so not built (run __graft_entry__.build())")
    return _abi.load(), _abi


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "mgcg.h")).read()
    return sorted(set(re.findall(r"\b(mgcg_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib, abi = _lib()
    names = _header_symbols()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.EXPORTS), set(names) ^ set(abi.EXPORTS)


def test_desc_validation_and_sizes():
    from paper_2311_05595_amd import api
    lib, abi = _lib()
    good = api.make_desc((24, 12, 12), nlevels=3)
    assert api.device_bytes(nel=(24, 12, 12), nlevels=3) > 0
    # odd element counts cannot be coarsened
    assert api.device_bytes(nel=(3, 2, 2), nlevels=2) == 0
    assert api.device_bytes(nel=(24, 12, 12), nrhs=5) == 0
    assert api.device_bytes(nel=(24, 12, 12), order=4) == 0
    assert api.device_bytes(nel=(4, 2, 2), order=2, nlevels=1) == 0
    assert api.device_bytes(nel=(4, 2, 2), order=3, nlevels=1) == 0
    # cubic elements: 192x192 element matrices (full, packed, by node for the
    # Gauss-Seidel smoother) and the packed sensitivity table for any nsub
    b3 = api.device_bytes(nel=(4, 2, 2), order=3, nlevels=2)
    assert b3 > 16 * 192 * 192 * 8
    assert api.device_bytes(nel=(4, 2, 2), order=3, nlevels=3) > 0
    assert api.device_bytes(nel=(4, 2, 2), order=3, nlevels=2, smoother="gauss-seidel") >= \
        b3 + 16 * 192 * 192 * 8
    # the serendipity family has degree 2 or 3
    assert api.device_bytes(nel=(4, 2, 2), order=2, nlevels=2, family="serendipity") > 0
    s3 = api.device_bytes(nel=(4, 2, 2), order=3, nlevels=2, family="serendipity")
    assert 0 < s3 < b3
    assert api.device_bytes(nel=(4, 2, 2), order=1, nlevels=2, family="serendipity") == 0
    assert api.device_bytes(nel=(4, 2, 2), order=2, nlevels=2, family=2) == 0
    # bytes grow with precision, nrhs and nsub
    b64 = api.device_bytes(nel=(32, 16, 16), nlevels=3)
    b2 = api.device_bytes(nel=(32, 16, 16), nlevels=3, nrhs=2)
    assert b2 > b64
    assert api.device_bytes(nel=(32, 16, 16), nlevels=3, nsub=2) > b64
    # the Gauss-Seidel smoother needs quadratic or cubic elements
    assert api.device_bytes(nel=(4, 2, 2), order=2, nlevels=2, smoother="gauss-seidel") > \
        api.device_bytes(nel=(4, 2, 2), order=2, nlevels=2)
    assert api.device_bytes(nel=(4, 2, 2), order=1, nlevels=2, smoother="gauss-seidel") == 0
    assert api.device_bytes(nel=(4, 2, 2), order=2, nlevels=2, smoother=2) == 0
    # a stencil finest level past the reduction buffer's 16,384 blocks of 64
    # nodes (161 x 81 x 81 nodes) is rejected up front, one within it is not
    assert api.device_bytes(nel=(160, 80, 80), nlevels=5, nsub=2) == 0
    assert api.device_bytes(nel=(128, 64, 64), nlevels=5, nsub=2) > 0
    del good


def test_problem_create_rejects_bad_input():
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError
    _lib()
    mask, f = W.make_problem("cantilever", 4, 2, 2, 1, 1)
    p = api.Problem((4, 2, 2), mask, f, nlevels=2)
    p.close()
    with pytest.raises(ValueError):
        api.Problem((4, 2, 2), mask[:-1], f, nlevels=2)
    bad = f.copy()
    bad[0, 5] = np.nan
    with pytest.raises(MGCGError):
        api.Problem((4, 2, 2), mask, bad, nlevels=2)
    with pytest.raises(MGCGError):
        api.Problem((4, 2, 2), mask, f, nlevels=2, omega=2.5)


def test_fused_launch_mode_eligibility():
    """The fused solve takes trilinear nsub = 1 FP64 Jacobi problems whose
    finest level fits the workgroup's LDS; others are refused up front (no
    device needed), and so is an empty or ineligible batch."""
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError
    _lib()
    mask, f = W.make_problem("cantilever", 8, 4, 4, 1, 2)
    ok = api.Problem((8, 4, 4), mask, f, nlevels=3)
    ok.set_launch_mode("fused")
    ok.set_launch_mode("eager")
    for kw in (dict(nsub=2), dict(precision="mixed"), dict(nlevels=1)):
        p = api.Problem((8, 4, 4), mask, f, **{**dict(nlevels=3), **kw})
        with pytest.raises(MGCGError):
            p.set_launch_mode("fused")
        with pytest.raises(MGCGError):
            api.solve_batch([ok, p])
        p.close()
    big_mask, big_f = W.make_problem("cantilever", 32, 16, 16, 1, 1)  # 9537 nodes
    big = api.Problem((32, 16, 16), big_mask, big_f, nlevels=4)
    with pytest.raises(MGCGError):
        big.set_launch_mode("fused")
    big.close()
    lib = ok._lib
    assert lib.mgcg_solve_batch(None, 1, 1e-8, 10, 0, None) != 0
    with pytest.raises(MGCGError):
        api.solve_batch([ok, ok])
    ok.close()


def test_admission_plan_respects_budget_and_order():
    from paper_2311_05595_amd import api
    _lib()
    adm = api.admission_plan(100, 10, 3, [30, 50, 20, 5])
    assert adm.tolist() == [True, True, False, False]  # 3rd would exceed, blocks the 4th
    adm = api.admission_plan(100, 0, 2, [10, 10, 10])
    assert adm.tolist() == [True, True, False]          # slots
    adm = api.admission_plan(100, 0, 4, [])
    assert adm.tolist() == []
    adm = api.admission_plan(100, 0, 4, [0, 0, 0])      # resident problems cost nothing
    assert adm.tolist() == [True, True, True]
    # a resident problem's next solve does not wait behind a request that
    # needs memory; memory-needing requests stay first-come-first-served
    adm = api.admission_plan(100, 80, 4, [50, 0, 10, 0])
    assert adm.tolist() == [False, True, False, True]
    big = np.iinfo(np.uint64).max                        # "cannot start now"
    adm = api.admission_plan(100, 0, 4, [big, 30, big, 0])
    assert adm.tolist() == [False, True, False, True]
    adm = api.admission_plan(100, 0, 1, [0, 0])         # slots still bound
    assert adm.tolist() == [True, False]
    # never over budget, whatever the queue
    rng = np.random.default_rng(0)
    for _ in range(200):
        q = rng.integers(0, 60, size=rng.integers(0, 10))
        used = int(rng.integers(0, 100))
        adm = api.admission_plan(100, used, int(rng.integers(0, 5)), q)
        assert used + int(q[adm].sum()) <= 100 or adm.sum() == 0
        # among requests needing memory, the admitted ones form a prefix
        need = adm[q > 0]
        k = int(need.sum())
        assert need[:k].all() and not need[k:].any()


def test_projection_desc_validation():
    """Projection sizes and the host-side checks (no device needed)."""
    from paper_2311_05595_amd import api
    _lib()
    b = api.proj_device_bytes((64, 32, 32), 4, 2, 1.5)
    # 1/omega per density cell, the weight-factor table (2 n d rmin + 2 entries)
    # and the gather tables of the tiled kernels (tens of kB)
    fixed = (64 * 32 * 32 * 64 + 26) * 8
    assert fixed + 8 * 100 * 16 < b <= fixed + 256 * 1024
    assert api.proj_device_bytes((2, 2, 2), 1, 1, 0.5) > 0
    # rejected: empty balls (nearest design centre 0.125 sqrt(3) away), bad sizes
    assert api.proj_device_bytes((1, 1, 1), 4, 2, 0.2) == 0
    assert api.proj_device_bytes((1, 1, 1), 4, 2, 0.2166) > 0
    assert api.proj_device_bytes((0, 1, 1), 1, 1, 1.0) == 0
    assert api.proj_device_bytes((1, 1, 1), 65, 1, 1.0) == 0
    assert api.proj_device_bytes((1, 1, 1), 1, 1, -1.0) == 0
    assert api.proj_device_bytes((1, 1, 1), 1, 1, float("nan")) == 0
    assert api.proj_device_bytes((1, 1, 1), 64, 64, 1.0) == 0  # 2 n d rmin > 4096
    assert api.proj_device_bytes((1 << 19, 1, 1), 4, 1, 1.0) == 0  # axis above 2^20 cells


def test_slp_step_control_matches_oracle():
    """mgcg_slp_decide (host) against the oracle's theta, merit and trust-region
    rules of Algorithm 2 over a seeded sequence of trial steps."""
    from paper_2311_05595_amd import api
    from oracle import slp
    _lib()
    rng = np.random.default_rng(12)
    ctrl = api.slp_ctrl(0.2, delta_min=1e-3, box_inf=1.0)
    delta, tmax, hist, k = 0.2, 1.0, [1.0], 0
    for _ in range(40):
        n = 20
        g = -rng.exponential(1.0, n)
        a = rng.uniform(0.5, 1.5, n)
        s = rng.uniform(-delta, delta, n)
        f0 = rng.uniform(1.0, 2.0)
        f1 = f0 - rng.uniform(-0.5, 1.0) * abs(g @ s)
        c0, c1 = rng.normal(0, 0.01), rng.normal(0, 0.01)
        gts, ats, sinf = float(g @ s), float(a @ s), float(np.abs(s).max())
        acc, th, ar, pr = api.slp_decide(ctrl, f0, f1, c0, c1, gts, ats, sinf)
        # oracle
        _, _, pf, po = slp.merit_reductions(1.0, f0, f1, g, s, c0, c1, a)
        th_o = slp.theta_update(k, hist, tmax, pf, po)
        ar_o, pr_o, _, _ = slp.merit_reductions(th_o, f0, f1, g, s, c0, c1, a)
        acc_o, delta_o = slp.trust_update(ar_o, pr_o, delta, sinf, 1.0, 1e-3)
        assert th == pytest.approx(th_o, rel=1e-13) and acc == acc_o
        assert ar == pytest.approx(ar_o, rel=1e-12, abs=1e-15)
        assert pr == pytest.approx(pr_o, rel=1e-12, abs=1e-15)
        assert ctrl.delta == pytest.approx(delta_o, rel=1e-14)
        delta = delta_o
        if acc_o:
            hist.append(th_o)
            tmax, k = 1.0, k + 1
        else:
            tmax = th_o
        assert ctrl.k == k
    assert api._abi.load().mgcg_lp_device_bytes(0) == 0
    assert api._abi.load().mgcg_lp_device_bytes(524288) > 524288 * 16


def test_new_entry_points_reject_bad_arguments_before_any_device_work():
    """Argument checks of the thresholding, fixing and fixed-LP entry points
    run on the host: NULL handles, bad geometry and bad thresholds return
    MGCG_EINVAL without touching a device."""
    import ctypes as C
    lib, abi = _lib()
    EINVAL = abi.MGCG_EINVAL
    null = C.c_void_p(0)
    d = C.c_double()
    it = C.c_int32()
    info = abi.mgcg_lp_info()
    assert lib.mgcg_lp_select_top(null, null, 0, null, 0) == EINVAL
    assert lib.mgcg_threshold_round(null, null, 0.05, 0.95, null, 0) == EINVAL
    assert lib.mgcg_angle_cos(null, null, null, C.byref(d), 0) == EINVAL
    assert lib.mgcg_heaviside(null, null, 1.0, null, C.byref(d), C.byref(it), 0) == EINVAL
    assert lib.mgcg_threshold_lagrangian(null, null, null, 0.3, 0.7, 89.9, null, C.byref(d), 0) == EINVAL
    assert lib.mgcg_lp_solve_fixed(null, null, null, null, null, 0.0, 0.1, 0.0, 1.0, null,
                                   C.byref(info), 0) == EINVAL
    assert lib.mgcg_fix_variables(None, null, null, null, null, null, None, 0) == EINVAL
    rho = np.zeros(8)
    buf = np.zeros(3 * 27, dtype=np.uint8)
    p = lambda a: C.c_void_p(a.ctypes.data)
    for desc in (abi.mgcg_fix_desc(2, 2, 2, 1, 1, 4, 1e-6, 0.9, 1e-6),      # order 4
                 abi.mgcg_fix_desc(0, 2, 2, 1, 1, 1, 1e-6, 0.9, 1e-6),      # empty mesh
                 abi.mgcg_fix_desc(2, 2, 2, 65, 1, 1, 1e-6, 0.9, 1e-6),     # n > 64
                 abi.mgcg_fix_desc(2, 2, 2, 1, 1, 1, float("nan"), 0.9, 1e-6)):
        assert lib.mgcg_fix_variables(C.byref(desc), p(rho), p(rho), p(buf), p(buf), p(buf),
                                      None, abi.MGCG_MEM_HOST) == EINVAL
    good = abi.mgcg_fix_desc(2, 2, 2, 1, 1, 1, 1e-6, 0.9, 1e-6)
    assert lib.mgcg_fix_variables(C.byref(good), p(rho), p(rho), p(buf), p(buf), p(buf), None,
                                  7) == EINVAL   # bad memory flag
    assert lib.mgcg_fix_variables(C.byref(good), null, p(rho), p(buf), p(buf), p(buf), None,
                                  abi.MGCG_MEM_HOST) == EINVAL


def test_context_accounting_without_a_device():
    """A context starts empty; a problem created in it counts as attached
    (no device memory until first use), and the context refuses to go while
    the problem lives."""
    import numpy as np
    import workloads as W
    from paper_2311_05595_amd import api
    lib, abi = _lib()
    ctx = api.Context(device=0, budget=1 << 20)
    assert ctx.usage() == (0, 1 << 20, 0)
    mask, f = W.make_problem("cantilever", 4, 2, 2, 1, 1)
    p = api.Problem((4, 2, 2), mask, f, nlevels=2, ctx=ctx)
    assert ctx.usage() == (0, 1 << 20, 1)
    assert lib.mgcg_ctx_destroy(ctx._h) == abi.MGCG_EINVAL
    p.close()
    assert ctx.usage() == (0, 1 << 20, 0)
    ctx.close()
    # null arguments
    assert lib.mgcg_problem_create_in(None, None, None, None, None) == abi.MGCG_EINVAL
    assert lib.mgcg_set_densities_f32(None, None, 0) == abi.MGCG_EINVAL
    assert lib.mgcg_ctx_usage(None, None, None, None) == abi.MGCG_EINVAL
    del np
