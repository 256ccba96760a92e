"""MGCG solver for SIMP linear elasticity on MI355X (gfx950).

Hand-written HIP kernels behind the C ABI of ``include/mgcg.h``; this package
is the thin Python binding (``api``), the autograd wrapper of the compliance
(``autograd``) and the in-tree build (``build``).
"""

from .api import Problem, Server, admission_plan, device_bytes, make_desc  # noqa: F401
from ._abi import load, MGCGError  # noqa: F401
