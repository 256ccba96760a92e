"""ctypes signatures of the C ABI (include/mgcg.h), same names, nothing else.

The library is the in-tree ``libmgcg.so`` built by ``paper_2311_05595_amd.build``.
Loading fails loudly when it is missing: there is no fallback path.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgcg.so")

MGCG_OK = 0
MGCG_ENOTCONV = 1
MGCG_EINVAL = -1
MGCG_ENOMEM = -2
MGCG_EBUDGET = -3
MGCG_EBREAKDOWN = -4
MGCG_EDEVICE = -5
MGCG_EAGAIN = -6
MGCG_ESTATE = -7

MGCG_FP64 = 0
MGCG_MIXED = 1
MGCG_MEM_HOST = 0
MGCG_MEM_DEVICE = 1

STATUS_NAMES = {0: "OK", 1: "ENOTCONV", -1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET",
                -4: "EBREAKDOWN", -5: "EDEVICE", -6: "EAGAIN", -7: "ESTATE"}


class mgcg_desc(C.Structure):
    _fields_ = [("nelx", C.c_int32), ("nely", C.c_int32), ("nelz", C.c_int32),
                ("order", C.c_int32), ("nsub", C.c_int32), ("nlevels", C.c_int32),
                ("nrhs", C.c_int32), ("precision", C.c_int32), ("pre", C.c_int32),
                ("post", C.c_int32), ("E0", C.c_double), ("Emin", C.c_double),
                ("nu", C.c_double), ("penal", C.c_double), ("omega", C.c_double),
                ("family", C.c_int32), ("smoother", C.c_int32)]


class mgcg_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32 * 4), ("rel_res", C.c_double * 4),
                ("replacements", C.c_int32), ("pad", C.c_int32), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double)]


class mgcg_proj_desc(C.Structure):
    _fields_ = [("nelx", C.c_int32), ("nely", C.c_int32), ("nelz", C.c_int32),
                ("nsub", C.c_int32), ("ndes", C.c_int32), ("pad", C.c_int32),
                ("rmin", C.c_double)]


class mgcg_lp_info(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("gts", C.c_double), ("ats", C.c_double),
                ("s_inf", C.c_double), ("budget", C.c_double), ("feasible", C.c_int32),
                ("pad", C.c_int32)]


class mgcg_slp_ctrl(C.Structure):
    _fields_ = [("delta", C.c_double), ("delta_min", C.c_double), ("box_inf", C.c_double),
                ("theta_max", C.c_double), ("theta_min_hist", C.c_double), ("N", C.c_double),
                ("k", C.c_int32), ("pad", C.c_int32)]


class mgcg_fix_desc(C.Structure):
    _fields_ = [("nelx", C.c_int32), ("nely", C.c_int32), ("nelz", C.c_int32),
                ("nsub", C.c_int32), ("ndes", C.c_int32), ("order", C.c_int32),
                ("rho_l", C.c_double), ("rho_u", C.c_double), ("eps_grad", C.c_double)]


class mgcg_fix_counts(C.Structure):
    _fields_ = [("void_elems", C.c_int64), ("solid_elems", C.c_int64),
                ("fixed_design", C.c_int64), ("suppressed_nodes", C.c_int64)]


EXPORTS = {
    # name: (restype, argtypes)
    "mgcg_last_error": (C.c_char_p, []),
    "mgcg_version": (C.c_int, []),
    "mgcg_problem_device_bytes": (C.c_size_t, [C.POINTER(mgcg_desc)]),
    "mgcg_problem_create": (C.c_int, [C.POINTER(mgcg_desc), C.c_void_p, C.c_void_p, C.c_int,
                                      C.POINTER(C.c_void_p)]),
    "mgcg_problem_destroy": (C.c_int, [C.c_void_p]),
    "mgcg_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgcg_get_stream": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "mgcg_set_launch_mode": (C.c_int, [C.c_void_p, C.c_int]),
    "mgcg_problem_allocate": (C.c_int, [C.c_void_p]),
    "mgcg_set_densities": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_set_densities_f32": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_size_t]),
    "mgcg_ctx_destroy": (C.c_int, [C.c_void_p]),
    "mgcg_ctx_usage": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                 C.POINTER(C.c_int32)]),
    "mgcg_problem_create_in": (C.c_int, [C.c_void_p, C.POINTER(mgcg_desc), C.c_void_p,
                                         C.c_void_p, C.POINTER(C.c_void_p)]),
    "mgcg_solve": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.POINTER(mgcg_info)]),
    "mgcg_solve_batch": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(mgcg_info)]),
    "mgcg_get_displacement": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_set_initial_guess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_compliance_sensitivity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_level_dims": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64)]),
    "mgcg_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_level_diag": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int]),
    "mgcg_restrict": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_prolong": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_precondition": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_coarse_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_set_kernel_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "mgcg_get_kernel_timing": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64)]),
    "mgcg_copy_bytes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "mgcg_server_create": (C.c_int, [C.c_int, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    "mgcg_server_destroy": (C.c_int, [C.c_void_p]),
    "mgcg_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                     C.c_int, C.c_int, C.POINTER(C.c_uint64)]),
    "mgcg_server_step": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "mgcg_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(mgcg_info),
                                   C.POINTER(C.c_double)]),
    "mgcg_server_release": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgcg_server_resident_bytes": (C.c_size_t, [C.c_void_p]),
    "mgcg_admission_plan": (C.c_int, [C.c_size_t, C.c_size_t, C.c_int, C.c_void_p, C.c_int,
                                      C.c_void_p]),
    "mgcg_proj_device_bytes": (C.c_size_t, [C.POINTER(mgcg_proj_desc)]),
    "mgcg_proj_create": (C.c_int, [C.POINTER(mgcg_proj_desc), C.c_int, C.POINTER(C.c_void_p)]),
    "mgcg_proj_destroy": (C.c_int, [C.c_void_p]),
    "mgcg_proj_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgcg_proj_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_proj_apply_transpose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "mgcg_lp_device_bytes": (C.c_size_t, [C.c_int64]),
    "mgcg_lp_create": (C.c_int, [C.c_int64, C.c_int, C.POINTER(C.c_void_p)]),
    "mgcg_lp_destroy": (C.c_int, [C.c_void_p]),
    "mgcg_lp_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mgcg_lp_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_void_p,
                                C.POINTER(mgcg_lp_info), C.c_int]),
    "mgcg_threshold_lagrangian": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                            C.c_double, C.c_double, C.c_void_p,
                                            C.POINTER(C.c_double), C.c_int]),
    "mgcg_lp_select_top": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int]),
    "mgcg_threshold_round": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                       C.c_void_p, C.c_int]),
    "mgcg_angle_cos": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                 C.c_int]),
    "mgcg_heaviside": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                 C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int]),
    "mgcg_fix_variables": (C.c_int, [C.POINTER(mgcg_fix_desc), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(mgcg_fix_counts), C.c_int]),
    "mgcg_fix_variables_noalloc": (C.c_int, [C.POINTER(mgcg_fix_desc), C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_void_p]),
    "mgcg_lp_solve_fixed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_void_p, C.POINTER(mgcg_lp_info), C.c_int]),
    "mgcg_slp_decide": (C.c_int, [C.POINTER(mgcg_slp_ctrl), C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
}

_lib = None


def load(path=None):
    """Load the library (once) and attach the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2311_05595_amd.build` "
            "(there is no CPU fallback)")
    # torch, when present, brings the HIP runtime first so that one runtime
    # serves both (same soname)
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    lib = C.CDLL(path, mode=C.RTLD_GLOBAL)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MGCGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, allow=(MGCG_OK,)):
    if code in allow:
        return code
    msg = load().mgcg_last_error()
    raise MGCGError(code, msg.decode() if msg else "")
