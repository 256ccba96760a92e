"""The fixing entry point that allocates nothing (static per-GPU scratch)
against the allocating one, through the C ABI: identical outputs on two calls
in a row, the second on a smaller mesh (the static scratch keeps the first
call's contents)."""

import ctypes as C

import numpy as np
import pytest

from helpers import need_gpu

pytestmark = pytest.mark.gpu


def _inputs(nel, n, d, order, seed):
    rng = np.random.default_rng(seed)
    nelx, nely, nelz = nel
    # blocks of void and solid with a noisy band, so that every rule binds
    rho = rng.uniform(0.0, 1.0, (nelz * n, nely * n, nelx * n))
    rho[:, :, : nelx * n // 3] = 1e-7
    rho[:, :, -(nelx * n // 3):] = 0.95
    # gradients inside the +-eps band almost everywhere, a few outside it
    grad = rng.normal(0.0, 2e-7, (nelz * d, nely * d, nelx * d))
    nn = (order * nelx + 1) * (order * nely + 1) * (order * nelz + 1)
    mask = np.zeros(3 * nn, dtype=np.uint8)
    mask[: 3 * (order * nelx + 1)] = 1
    return rho.ravel(), grad.ravel(), mask


def _call_both(lib, abi, nel, n, d, order, seed):
    import torch
    desc = abi.mgcg_fix_desc(nel[0], nel[1], nel[2], n, d, order, 1e-6, 0.9, 1e-6)
    rho, grad, mask = _inputs(nel, n, d, order, seed)
    dev = torch.device("cuda:0")
    t_rho = torch.tensor(rho, dtype=torch.float64, device=dev)
    t_grad = torch.tensor(grad, dtype=torch.float64, device=dev)
    nelt = nel[0] * nel[1] * nel[2]
    outs = []
    for noalloc in (False, True):
        kind = torch.full((nelt,), 77, dtype=torch.uint8, device=dev)
        des = torch.full((nelt * d ** 3,), 77, dtype=torch.uint8, device=dev)
        m = torch.tensor(mask, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        if noalloc:
            cnt = torch.full((4,), -1, dtype=torch.int64, device=dev)
            st = torch.cuda.current_stream().cuda_stream
            rc = lib.mgcg_fix_variables_noalloc(C.byref(desc), C.c_void_p(t_rho.data_ptr()),
                                                C.c_void_p(t_grad.data_ptr()),
                                                C.c_void_p(kind.data_ptr()),
                                                C.c_void_p(des.data_ptr()),
                                                C.c_void_p(m.data_ptr()),
                                                C.c_void_p(cnt.data_ptr()), C.c_void_p(st))
            assert rc == 0, lib.mgcg_last_error()
            torch.cuda.synchronize()
            counts = cnt.cpu().numpy().tolist()
        else:
            c = abi.mgcg_fix_counts()
            rc = lib.mgcg_fix_variables(C.byref(desc), C.c_void_p(t_rho.data_ptr()),
                                        C.c_void_p(t_grad.data_ptr()), C.c_void_p(kind.data_ptr()),
                                        C.c_void_p(des.data_ptr()), C.c_void_p(m.data_ptr()),
                                        C.byref(c), abi.MGCG_MEM_DEVICE)
            assert rc == 0, lib.mgcg_last_error()
            counts = [c.void_elems, c.solid_elems, c.fixed_design, c.suppressed_nodes]
        outs.append((kind.cpu().numpy(), des.cpu().numpy(), m.cpu().numpy(), counts))
    return outs


def test_noalloc_fixing_equals_allocating_one():
    need_gpu()
    from paper_2311_05595_amd import _abi as abi
    lib = abi.load()
    # a larger call, then a smaller one on the same static scratch
    for nel, n, d, order, seed in [((40, 20, 16), 4, 2, 2, 1), ((12, 6, 6), 2, 1, 1, 2)]:
        ref, got = _call_both(lib, abi, nel, n, d, order, seed)
        for a, b in zip(ref[:3], got[:3]):
            assert np.array_equal(a, b)
        assert ref[3] == got[3]
        assert ref[3][0] > 0 and ref[3][1] > 0 and ref[3][3] > 0  # every count non-trivial


def test_noalloc_fixing_rejects_oversized_mesh():
    need_gpu()
    from paper_2311_05595_amd import _abi as abi
    lib = abi.load()
    # 40M elements need ~40 MB of scratch, above the 16 MiB limit
    desc = abi.mgcg_fix_desc(400, 400, 250, 1, 1, 1, 1e-6, 0.9, 1e-6)
    dummy = C.c_void_p(8)
    rc = lib.mgcg_fix_variables_noalloc(C.byref(desc), dummy, dummy, dummy, dummy, dummy, dummy,
                                        C.c_void_p(0))
    assert rc == abi.MGCG_EINVAL
    assert b"scratch" in lib.mgcg_last_error()
