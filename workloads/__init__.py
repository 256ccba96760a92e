"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This package holds no arithmetic of the solve, the operator or the sensitivity:
only problem *data* — density fields, supports (fixed-DOF masks) and nodal load
vectors — built from seeds.  The HIP library and the CPU oracle both receive
these arrays as inputs.

Conventions (shared by every consumer):

* node lattice of a mesh of ``nelx x nely x nelz`` elements of order ``p``:
  ``NX = p*nelx + 1`` (same for y, z); node index ``i + NX*(j + NY*k)``, x fastest;
* DOF index ``3*node + c`` with c = 0, 1, 2 for the x, y, z components;
* density lattice of ``nsub`` sub-elements per axis per element:
  C-order array of shape ``(nsub*nelz, nsub*nely, nsub*nelx)``;
* y is the vertical axis (loads act in -y); elements are unit cubes.
"""

from .fields import uniform_field, gaussian_random_field, perturb, solid_at_supports_and_loads
from .loads import (
    node_dims,
    cantilever_bcs,
    mbb_bcs,
    torsion_bcs,
    pressure_load,
    make_problem,
)
from .configs import CONFIGS, config

__all__ = [
    "uniform_field",
    "gaussian_random_field",
    "perturb",
    "solid_at_supports_and_loads",
    "node_dims",
    "cantilever_bcs",
    "mbb_bcs",
    "torsion_bcs",
    "pressure_load",
    "make_problem",
    "CONFIGS",
    "config",
]
