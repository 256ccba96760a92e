"""Python binding over the C ABI: argument marshalling only.

Every computation runs in the HIP library; numpy arrays are passed as host
pointers, CUDA/HIP torch tensors as device pointers (FP64, contiguous) on the
current torch stream.
"""

import ctypes as C
import math

import numpy as np

from . import _abi
from ._abi import (MGCG_EAGAIN, MGCG_ENOTCONV, MGCG_FP64, MGCG_MEM_DEVICE, MGCG_MEM_HOST,
                   MGCG_MIXED, MGCG_OK, check, load, mgcg_desc, mgcg_info)

_PREC = {"fp64": MGCG_FP64, "mixed": MGCG_MIXED}


def _torch():
    import torch
    return torch


def _is_device_tensor(a):
    try:
        torch = _torch()
    except Exception:
        return False
    return isinstance(a, torch.Tensor) and a.is_cuda


def _is_float32(a):
    if _is_device_tensor(a):
        return a.dtype == _torch().float32
    return getattr(a, "dtype", None) == np.float32


def _ptr(a, dtype=np.float64):
    """(pointer, mem flag, keep-alive) for a numpy array or a device tensor."""
    if _is_device_tensor(a):
        torch = _torch()
        want = torch.float32 if dtype == np.float32 else torch.float64
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"device tensors must be contiguous {want}")
        return C.c_void_p(a.data_ptr()), MGCG_MEM_DEVICE, a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return C.c_void_p(arr.ctypes.data), MGCG_MEM_HOST, arr


def _inputs_ready(mem):
    """For calls that run on the null stream: unless torch's current stream
    is the null stream itself, finish the torch work that produced a device
    input before handing it over."""
    if mem == MGCG_MEM_DEVICE:
        cur = _torch().cuda.current_stream()
        if cur.cuda_stream != 0:
            cur.synchronize()


def _order_after_torch(mem, stream_ptr):
    """A device input produced on torch's current stream is read on the
    stream `stream_ptr` (a hipStream_t): nothing to do when they are the same
    stream; otherwise that stream waits for torch's on the device (an event),
    without a host synchronisation."""
    if mem != MGCG_MEM_DEVICE:
        return
    torch = _torch()
    cur = torch.cuda.current_stream()
    if cur.cuda_stream == stream_ptr:
        return
    torch.cuda.ExternalStream(stream_ptr, device=cur.device).wait_stream(cur)


def _warm(w):
    """warm_start argument: True / "scaled" (the previous solution scaled by
    the energy-minimising factor), "plain" (as it is), False / "cold"."""
    if isinstance(w, str):
        return {"cold": 0, "scaled": 1, "plain": 2}[w]
    return 1 if w else 0


def _info(i):
    return dict(status=i.status, iters=list(i.iters), rel_res=list(i.rel_res),
                replacements=i.replacements, t_setup_ms=i.t_setup_ms, t_solve_ms=i.t_solve_ms)


def solve_batch(problems, rtol=1e-8, maxit=1000, warm_start=True, allow_notconv=False):
    """Solve several small problems in one launch (mgcg_solve_batch): each
    must fit the fused solve and have its densities set.  Returns their info
    dicts in order."""
    problems = list(problems)
    if not problems:
        return []
    lib = problems[0]._lib
    hs = (C.c_void_p * len(problems))(*[p._h.value for p in problems])
    infos = (mgcg_info * len(problems))()
    allow = (MGCG_OK, MGCG_ENOTCONV) if allow_notconv else (MGCG_OK,)
    check(lib.mgcg_solve_batch(hs, len(problems), rtol, maxit, _warm(warm_start), infos), allow)
    return [_info(i) for i in infos]


_FAMILY = {"lagrange": 0, "serendipity": 1}


_SMOOTHER = {"jacobi": 0, "gauss-seidel": 1}


def make_desc(nel, order=1, nsub=1, nlevels=3, nrhs=1, precision="fp64", E0=1.0, Emin=1e-9,
              nu=0.3, penal=3.0, omega=0.6, pre=1, post=1, family="lagrange", smoother="jacobi"):
    return mgcg_desc(nel[0], nel[1], nel[2], order, nsub, nlevels, nrhs,
                     _PREC[precision] if isinstance(precision, str) else int(precision),
                     pre, post, E0, Emin, nu, penal, omega,
                     _FAMILY[family] if isinstance(family, str) else int(family),
                     _SMOOTHER[smoother] if isinstance(smoother, str) else int(smoother))


def device_bytes(**kw):
    return load().mgcg_problem_device_bytes(C.byref(make_desc(**kw)))


class Context:
    """A device and an HBM budget (bytes; 0: none) shared by the problems
    created with ctx=this context (mgcg_ctx_* in include/mgcg.h)."""

    def __init__(self, device=0, budget=0):
        self._lib = load()
        h = C.c_void_p()
        check(self._lib.mgcg_ctx_create(C.byref(h), device, budget))
        self._h = h

    def usage(self):
        """(bytes charged, budget, live problems)."""
        a, b, n = C.c_size_t(), C.c_size_t(), C.c_int32()
        check(self._lib.mgcg_ctx_usage(self._h, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            check(self._lib.mgcg_ctx_destroy(self._h))
            self._h = None


class Problem:
    """One equilibrium problem K(rho) u = f (all load cases) on one GPU."""

    def __init__(self, nel, mask, f, order=1, nsub=1, nlevels=3, precision="fp64", E0=1.0,
                 Emin=1e-9, nu=0.3, penal=3.0, omega=0.6, pre=1, post=1, device=0,
                 family="lagrange", smoother="jacobi", ctx=None):
        lib = load()
        f = np.atleast_2d(np.ascontiguousarray(f, dtype=np.float64))
        self.nrhs = f.shape[0]
        self.nel = tuple(nel)
        self.order, self.nsub, self.nlevels = order, nsub, nlevels
        self.desc = make_desc(nel, order, nsub, nlevels, self.nrhs, precision, E0, Emin, nu,
                              penal, omega, pre, post, family, smoother)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.f = f
        dims = [order * n + 1 for n in nel]
        self.ndof = 3 * dims[0] * dims[1] * dims[2]
        self.nrho = nel[0] * nel[1] * nel[2] * nsub ** 3
        if self.mask.size != self.ndof or f.shape[1] != self.ndof:
            raise ValueError("mask/f size does not match the mesh")
        h = C.c_void_p()
        if ctx is None:
            check(lib.mgcg_problem_create(C.byref(self.desc), C.c_void_p(self.mask.ctypes.data),
                                          C.c_void_p(f.ctypes.data), device, C.byref(h)))
        else:
            check(lib.mgcg_problem_create_in(ctx._h, C.byref(self.desc),
                                             C.c_void_p(self.mask.ctypes.data),
                                             C.c_void_p(f.ctypes.data), C.byref(h)))
        self._h = h
        self._lib = lib

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mgcg_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self):
        return self._lib.mgcg_problem_device_bytes(C.byref(self.desc))

    def allocate(self):
        check(self._lib.mgcg_problem_allocate(self._h))

    def set_stream(self, stream=None):
        """stream: a torch.cuda.Stream, a raw hipStream_t (int) or None."""
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        check(self._lib.mgcg_set_stream(self._h, C.c_void_p(stream or 0)))

    def use_torch_stream(self):
        self.set_stream(_torch().cuda.current_stream().cuda_stream)

    def set_launch_mode(self, mode):
        """"eager", "graph" (replay one captured PCG iteration) or "fused"
        (the whole solve in one launch, a workgroup per load case; small
        trilinear FP64 problems only)."""
        check(self._lib.mgcg_set_launch_mode(self._h, {"eager": 0, "graph": 1, "fused": 2}[mode]))

    def stream(self):
        """The hipStream_t (int) the problem's work runs on."""
        s = C.c_void_p()
        check(self._lib.mgcg_get_stream(self._h, C.byref(s)))
        return s.value or 0

    def set_densities(self, rho):
        """rho: [n_rho] float64, or float32 (converted to FP64 by the
        library), as a numpy array or a contiguous device tensor."""
        f32 = _is_float32(rho)
        p, mem, keep = _ptr(rho, np.float32 if f32 else np.float64)
        _order_after_torch(mem, self.stream() if mem == MGCG_MEM_DEVICE else 0)
        if (keep.numel() if mem == MGCG_MEM_DEVICE else keep.size) != self.nrho:
            raise ValueError("density count does not match the mesh")
        if f32:
            check(self._lib.mgcg_set_densities_f32(self._h, p, mem))
        else:
            check(self._lib.mgcg_set_densities(self._h, p, mem))

    def solve(self, rtol=1e-8, maxit=1000, warm_start=True, allow_notconv=False):
        info = mgcg_info()
        allow = (MGCG_OK, MGCG_ENOTCONV) if allow_notconv else (MGCG_OK,)
        check(self._lib.mgcg_solve(self._h, rtol, maxit, _warm(warm_start), C.byref(info)),
              allow)
        return _info(info)

    def displacement(self, out=None):
        if out is None:
            out = np.empty((self.nrhs, self.ndof))
        p, mem, _ = _ptr(out) if _is_device_tensor(out) else (C.c_void_p(out.ctypes.data), MGCG_MEM_HOST, out)
        check(self._lib.mgcg_get_displacement(self._h, p, mem))
        return out

    def set_initial_guess(self, u):
        p, mem, _k = _ptr(u)
        _order_after_torch(mem, self.stream() if mem == MGCG_MEM_DEVICE else 0)
        check(self._lib.mgcg_set_initial_guess(self._h, p, mem))

    def compliance_sensitivity(self, dc_out=None, want_dc=True):
        """Returns (c per load case + total [nrhs+1] numpy, dc or None)."""
        c = np.zeros(self.nrhs + 1)
        if want_dc and dc_out is None:
            dc_out = np.empty(self.nrho)
        if dc_out is None:
            dp, mem = C.c_void_p(0), MGCG_MEM_HOST
        elif _is_device_tensor(dc_out):
            dp, mem, _ = _ptr(dc_out)
        else:
            dp, mem = C.c_void_p(dc_out.ctypes.data), MGCG_MEM_HOST
        check(self._lib.mgcg_compliance_sensitivity(self._h, C.c_void_p(c.ctypes.data), dp, mem))
        return c, dc_out

    # ---- inspection (parity tests) ----
    def level_dims(self, level):
        d = (C.c_int32 * 3)()
        n = C.c_int64()
        check(self._lib.mgcg_level_dims(self._h, level, d, C.byref(n)))
        return tuple(d), n.value

    def _vec_op(self, fn, level, x, out_len, *extra):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(out_len)
        check(fn(self._h, level, *extra, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data),
                 MGCG_MEM_HOST))
        return y

    def apply(self, level, x, precision="fp64"):
        n = self.level_dims(level)[1] * self.nrhs
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
        y = np.empty(n)
        check(self._lib.mgcg_apply(self._h, level, _PREC[precision], C.c_void_p(x.ctypes.data),
                                   C.c_void_p(y.ctypes.data), MGCG_MEM_HOST))
        return y.reshape(self.nrhs, -1)

    def diag(self, level):
        n = self.level_dims(level)[1]
        y = np.empty(n)
        check(self._lib.mgcg_level_diag(self._h, level, C.c_void_p(y.ctypes.data), MGCG_MEM_HOST))
        return y

    def restrict(self, level, fine):
        nc = self.level_dims(level + 1)[1] * self.nrhs
        fine = np.ascontiguousarray(fine, dtype=np.float64).reshape(-1)
        out = np.empty(nc)
        check(self._lib.mgcg_restrict(self._h, level, C.c_void_p(fine.ctypes.data),
                                      C.c_void_p(out.ctypes.data), MGCG_MEM_HOST))
        return out.reshape(self.nrhs, -1)

    def prolong(self, level, coarse):
        nf = self.level_dims(level)[1] * self.nrhs
        coarse = np.ascontiguousarray(coarse, dtype=np.float64).reshape(-1)
        out = np.empty(nf)
        check(self._lib.mgcg_prolong(self._h, level, C.c_void_p(coarse.ctypes.data),
                                     C.c_void_p(out.ctypes.data), MGCG_MEM_HOST))
        return out.reshape(self.nrhs, -1)

    def precondition(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
        z = np.empty_like(r)
        check(self._lib.mgcg_precondition(self._h, C.c_void_p(r.ctypes.data),
                                          C.c_void_p(z.ctypes.data), MGCG_MEM_HOST))
        return z.reshape(self.nrhs, -1)

    def coarse_solve(self, b):
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        x = np.empty_like(b)
        check(self._lib.mgcg_coarse_solve(self._h, C.c_void_p(b.ctypes.data),
                                          C.c_void_p(x.ctypes.data), MGCG_MEM_HOST))
        return x.reshape(self.nrhs, -1)

    def set_kernel_timing(self, kernel=0, enable=True):
        check(self._lib.mgcg_set_kernel_timing(self._h, kernel + 1 if enable else 0))

    def kernel_timing(self, kernel=0):
        ms = C.c_double()
        n = C.c_int64()
        check(self._lib.mgcg_get_kernel_timing(self._h, kernel, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def copy_bytes(self, src_ptr, dst_ptr, nbytes):
        check(self._lib.mgcg_copy_bytes(self._h, C.c_void_p(src_ptr), C.c_void_p(dst_ptr), nbytes))


def admission_plan(budget, in_use, free_slots, queue_bytes):
    lib = load()
    q = np.ascontiguousarray(queue_bytes, dtype=np.uint64)
    adm = np.zeros(len(q), dtype=np.uint8)
    n = lib.mgcg_admission_plan(budget, in_use, free_slots, C.c_void_p(q.ctypes.data), len(q),
                                C.c_void_p(adm.ctypes.data))
    if n < 0:
        check(n)
    return adm.astype(bool)


class Server:
    """Continuous-batching server (see mgcg_server_* in include/mgcg.h)."""

    def __init__(self, budget_bytes, max_slots=8, device=0):
        lib = load()
        h = C.c_void_p()
        check(lib.mgcg_server_create(device, int(budget_bytes), int(max_slots), C.byref(h)))
        self._h, self._lib = h, lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mgcg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, problem, rho, rtol=1e-8, maxit=1000, warm_start=True):
        """rho: a numpy array, or a contiguous float64 device tensor (copied
        on the device, in order after torch's current stream)."""
        p, mem, keep = _ptr(rho)
        if (keep.numel() if mem == MGCG_MEM_DEVICE else keep.size) != problem.nrho:
            raise ValueError("density count does not match the mesh")
        if mem == MGCG_MEM_DEVICE:
            _order_after_torch(mem, problem.stream())
        t = C.c_uint64()
        check(self._lib.mgcg_server_submit(self._h, problem.handle, p, mem, rtol, maxit,
                                           _warm(warm_start), C.byref(t)))
        return t.value

    def step(self):
        a, q = C.c_int(), C.c_int()
        check(self._lib.mgcg_server_step(self._h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def poll(self, ticket):
        """None while running; else (status, info dict, latency ms)."""
        info = mgcg_info()
        lat = C.c_double()
        st = self._lib.mgcg_server_poll(self._h, ticket, C.byref(info), C.byref(lat))
        if st == MGCG_EAGAIN:
            return None
        return st, _info(info), lat.value

    def release(self, problem):
        check(self._lib.mgcg_server_release(self._h, problem.handle))

    def resident_bytes(self):
        return self._lib.mgcg_server_resident_bytes(self._h)


def make_proj_desc(nel, nsub, ndes, rmin):
    return _abi.mgcg_proj_desc(int(nel[0]), int(nel[1]), int(nel[2]), int(nsub), int(ndes), 0,
                               float(rmin))


def proj_device_bytes(nel, nsub, ndes, rmin):
    return load().mgcg_proj_device_bytes(C.byref(make_proj_desc(nel, nsub, ndes, rmin)))


class Projection:
    """Design variables -> densities, rho = W x, and the chain rule g_x = W^T g
    (mgcg_proj_* in include/mgcg.h).  Vectors: numpy arrays (host) or
    contiguous float64 device tensors (run on the current torch stream)."""

    def __init__(self, nel, nsub, ndes, rmin, device=0):
        lib = load()
        self.nel, self.nsub, self.ndes, self.rmin = tuple(nel), int(nsub), int(ndes), float(rmin)
        self.desc = make_proj_desc(nel, nsub, ndes, rmin)
        h = C.c_void_p()
        check(lib.mgcg_proj_create(C.byref(self.desc), int(device), C.byref(h)))
        self._h, self._lib = h, lib
        self.nrho = int(np.prod(nel)) * self.nsub ** 3
        self.nx = int(np.prod(nel)) * self.ndes ** 3

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mgcg_proj_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        check(self._lib.mgcg_proj_set_stream(self._h, C.c_void_p(stream or 0)))

    def _run(self, fn, v, nin, nout, out):
        p, mem, keep = _ptr(v)
        if (keep.numel() if mem == MGCG_MEM_DEVICE else keep.size) != nin:
            raise ValueError("vector length does not match the lattice")
        if mem == MGCG_MEM_DEVICE:
            torch = _torch()
            # torch's current stream, the default (null) stream included
            cur = torch.cuda.current_stream().cuda_stream
            if cur != getattr(self, "_stream", 0):
                self.set_stream(cur)
                self._stream = cur
            if out is None:
                out = torch.empty(nout, dtype=torch.float64, device=keep.device)
            q, _, _ = _ptr(out)
        else:
            out = np.empty(nout) if out is None else out
            q = C.c_void_p(out.ctypes.data)
        check(fn(self._h, p, q, mem))
        return out

    def apply(self, x, out=None):
        return self._run(self._lib.mgcg_proj_apply, x, self.nx, self.nrho, out)

    def apply_transpose(self, g, out=None):
        return self._run(self._lib.mgcg_proj_apply_transpose, g, self.nrho, self.nx, out)


class LP:
    """The LP subproblem of the SLP step (mgcg_lp_* in include/mgcg.h) for n
    variables.  solve() returns (s, info dict); vectors are numpy arrays or
    contiguous float64 device tensors (then run on the current torch stream)."""

    def __init__(self, n, device=0):
        lib = load()
        h = C.c_void_p()
        check(lib.mgcg_lp_create(int(n), int(device), C.byref(h)))
        self._h, self._lib, self.n = h, lib, int(n)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mgcg_lp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vectors(self, *vs):
        """Pointers of equal-length vectors, their memory kind, keep-alives."""
        ps, keep = [], []
        mem = None
        for v in vs:
            p, m, k = _ptr(v)
            if mem is not None and m != mem:
                raise ValueError("mixed host and device vectors")
            mem = m
            if (k.numel() if m == MGCG_MEM_DEVICE else k.size) != self.n:
                raise ValueError("vector length does not match the LP size")
            ps.append(p)
            keep.append(k)
        if mem == MGCG_MEM_DEVICE:
            torch = _torch()
            cur = torch.cuda.current_stream().cuda_stream
            if cur != getattr(self, "_stream", 0):
                check(self._lib.mgcg_lp_set_stream(self._h, C.c_void_p(cur)))
                self._stream = cur
        return ps, mem, keep

    def _out(self, out, mem, like):
        if mem == MGCG_MEM_DEVICE:
            torch = _torch()
            if out is None:
                out = torch.empty(self.n, dtype=torch.float64, device=like.device)
            return out, C.c_void_p(out.data_ptr())
        out = np.empty(self.n) if out is None else out
        return out, C.c_void_p(out.ctypes.data)

    def solve(self, g, a, x, b, delta, x_l=0.0, x_u=1.0, out=None, fixed=None):
        """fixed: optional uint8 mask (numpy or device tensor, like g) of
        variables held at s = 0 (Sec. 6.1)."""
        (pg, pa, px), mem, keep = self._vectors(g, a, x)
        out, ps = self._out(out, mem, keep[0])
        info = _abi.mgcg_lp_info()
        if fixed is None:
            check(self._lib.mgcg_lp_solve(self._h, pg, pa, px, float(b), float(delta),
                                          float(x_l), float(x_u), ps, C.byref(info), mem))
        else:
            if _is_device_tensor(fixed):
                if fixed.dtype != _torch().uint8 or not fixed.is_contiguous():
                    raise TypeError("device fixed flags must be contiguous uint8")
                pf, mem_f, kf = C.c_void_p(fixed.data_ptr()), MGCG_MEM_DEVICE, fixed
            else:
                pf, mem_f, kf = _ptr(fixed, dtype=np.uint8)
            if mem_f != mem or (kf.numel() if mem == MGCG_MEM_DEVICE else kf.size) != self.n:
                raise ValueError("fixed must be n flags in the vectors' memory")
            check(self._lib.mgcg_lp_solve_fixed(self._h, pg, pa, px, pf, float(b), float(delta),
                                                float(x_l), float(x_u), ps, C.byref(info), mem))
        return out, {"lambda": info.lambda_, "gts": info.gts, "ats": info.ats,
                     "s_inf": info.s_inf, "budget": info.budget,
                     "feasible": bool(info.feasible)}

    def select_top(self, v, k, out=None):
        """1 for the k largest values (equal values in index order), 0 else."""
        (pv,), mem, keep = self._vectors(v)
        out, po = self._out(out, mem, keep[0])
        check(self._lib.mgcg_lp_select_top(self._h, pv, int(k), po, mem))
        return out

    def density_threshold(self, rho, vfrac, out=None):
        """The strategy based on the density values (Sec. 5.1): the
        floor(vfrac n) highest densities to 1, the rest to 0."""
        return self.select_top(rho, int(math.floor(vfrac * self.n)), out)

    def pre_round(self, rho, lo=0.05, hi=0.95, out=None):
        (pr,), mem, keep = self._vectors(rho)
        out, po = self._out(out, mem, keep[0])
        check(self._lib.mgcg_threshold_round(self._h, pr, float(lo), float(hi), po, mem))
        return out

    def angle_cos(self, gL, d):
        """-gL^T d / (|gL| |d|) (the angle condition of Sec. 5.2)."""
        (pg, pd), mem, _ = self._vectors(gL, d)
        c = C.c_double()
        check(self._lib.mgcg_angle_cos(self._h, pg, pd, C.byref(c), mem))
        return c.value

    def lagrangian_threshold(self, rho, gL, v_u=0.3, v_l=0.7, theta_max_deg=89.9, out=None):
        """The strategy based on the gradient of the Lagrangian (Sec. 5.2) on
        pre-rounded densities; returns (rho~, alpha~)."""
        (pr, pg), mem, keep = self._vectors(rho, gL)
        out, po = self._out(out, mem, keep[0])
        a = C.c_double()
        check(self._lib.mgcg_threshold_lagrangian(self._h, pr, pg, float(v_u), float(v_l),
                                                  float(theta_max_deg), po, C.byref(a), mem))
        return out, a.value

    def heaviside(self, rho, beta, out=None):
        """Smooth Heaviside projection with the volume-preserving threshold
        (Sec. 5.4); returns (h, eta, Newton iterations)."""
        (pr,), mem, keep = self._vectors(rho)
        out, po = self._out(out, mem, keep[0])
        eta, it = C.c_double(), C.c_int32()
        check(self._lib.mgcg_heaviside(self._h, pr, float(beta), po, C.byref(eta), C.byref(it),
                                       mem))
        return out, eta.value, it.value


def slp_ctrl(delta0, delta_min=1e-3, box_inf=1.0, N=1e6):
    """Initial step-control state of Algorithm 2."""
    return _abi.mgcg_slp_ctrl(float(delta0), float(delta_min), float(box_inf), 1.0, 1.0,
                              float(N), 0, 0)


def slp_decide(ctrl, f0, f1, c0, c1, gts, ats, s_inf):
    """One accept/reject decision of Algorithm 2 (updates ctrl in place);
    returns (accepted, theta, A_red, P_red)."""
    th, ar, pr = C.c_double(), C.c_double(), C.c_double()
    r = load().mgcg_slp_decide(C.byref(ctrl), f0, f1, c0, c1, gts, ats, s_inf, C.byref(th),
                               C.byref(ar), C.byref(pr))
    if r < 0:
        check(r)
    return bool(r), th.value, ar.value, pr.value


def fix_variables(nel, nsub, ndes, order, rho, grad_x, dof_mask, rho_l=1e-6, rho_u=0.9,
                  eps_grad=1e-6):
    """Variables fixed before the degree is raised (Sec. 6.1, mgcg_fix_variables).

    rho and grad_x: numpy arrays or contiguous float64 device tensors of the
    density and design lattices; dof_mask: the supports' uint8 mask of the
    lattice of degree `order` (host or device like rho), updated in place.
    Returns (elem_kind, design_fixed, dof_mask, counts dict)."""
    desc = _abi.mgcg_fix_desc(int(nel[0]), int(nel[1]), int(nel[2]), int(nsub), int(ndes),
                              int(order), float(rho_l), float(rho_u), float(eps_grad))
    pr, mem, kr = _ptr(rho)
    pg, mem_g, _ = _ptr(grad_x)
    if mem_g != mem:
        raise ValueError("mixed host and device arrays")
    nelt = int(nel[0]) * int(nel[1]) * int(nel[2])
    nx = nelt * int(ndes) ** 3
    nn = (order * nel[0] + 1) * (order * nel[1] + 1) * (order * nel[2] + 1)
    if mem == MGCG_MEM_DEVICE:
        torch = _torch()
        if dof_mask.dtype != torch.uint8 or not dof_mask.is_contiguous() or dof_mask.numel() != 3 * nn:
            raise ValueError("dof_mask must be a contiguous uint8 tensor of 3 entries per node")
        _inputs_ready(mem)
        kind = torch.empty(nelt, dtype=torch.uint8, device=kr.device)
        des = torch.empty(nx, dtype=torch.uint8, device=kr.device)
        pk, pd, pm = (C.c_void_p(t.data_ptr()) for t in (kind, des, dof_mask))
    else:
        if not (isinstance(dof_mask, np.ndarray) and dof_mask.dtype == np.uint8 and
                dof_mask.flags.c_contiguous and dof_mask.size == 3 * nn):
            raise ValueError("dof_mask must be a contiguous uint8 array of 3 entries per node")
        kind = np.empty(nelt, dtype=np.uint8)
        des = np.empty(nx, dtype=np.uint8)
        pk, pd, pm = (C.c_void_p(a.ctypes.data) for a in (kind, des, dof_mask))
    cnt = _abi.mgcg_fix_counts()
    check(load().mgcg_fix_variables(C.byref(desc), pr, pg, pk, pd, pm, C.byref(cnt), mem))
    return kind, des, dof_mask, {"void_elems": cnt.void_elems, "solid_elems": cnt.solid_elems,
                                 "fixed_design": cnt.fixed_design,
                                 "suppressed_nodes": cnt.suppressed_nodes}


__all__ = ["Problem", "Server", "Projection", "LP", "slp_ctrl", "slp_decide", "fix_variables", "admission_plan", "device_bytes", "make_desc",
           "make_proj_desc", "proj_device_bytes", "_abi"]
