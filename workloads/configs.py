"""The synthetic workloads of the MGCG hot path (sizes, material, solver
settings and seeds), plus the served request mix.

Material of every workload: E0 = 1, Emin = 1e-9, nu = 0.3, SIMP p = 3
(the paper's values for its adaptive runs; unit cube elements).
"""

import numpy as np

from .fields import uniform_field, gaussian_random_field, perturb, solid_at_supports_and_loads
from .loads import make_problem

MATERIAL = dict(E0=1.0, Emin=1e-9, nu=0.3, penal=3.0)

CONFIGS = {
    # plain FP64, single resolution, small (the oracle finishes it in seconds)
    "c1": dict(name="cantilever Q1 24x12x12 n=1 fp64", kind="cantilever",
               nel=(24, 12, 12), order=1, nsub=1, nlevels=3, nrhs=1,
               precision="fp64", omega=0.6, pre=1, post=1,
               field="uniform", seed=1),
    # plain FP64 at scale, warm-started over 10 SLP-like perturbations
    "c2": dict(name="cantilever Q1 96x48x48 n=1 fp64", kind="cantilever",
               nel=(96, 48, 48), order=1, nsub=1, nlevels=5, nrhs=1,
               precision="fp64", omega=0.6, pre=1, post=1,
               field="grf", seed=2, perturb_seeds=list(range(2001, 2011))),
    # multiresolution n=4 + mixed precision + adjoint
    "c3": dict(name="cantilever Q1 64x32x32 n=4 mixed", kind="cantilever",
               nel=(64, 32, 32), order=1, nsub=4, nlevels=5, nrhs=1,
               precision="mixed", omega=0.6, pre=1, post=1,
               field="grf", seed=3),
    # quadratic elements, n=4, two load cases
    "c4": dict(name="cantilever Q2 48x24x24 n=4 2rhs mixed", kind="cantilever",
               nel=(48, 24, 24), order=2, nsub=4, nlevels=5, nrhs=2,
               precision="mixed", omega=0.6, pre=1, post=1,
               field="grf", seed=4),
    # the quadratic serendipity element on the c4 mesh, tip load only (the
    # top pressure's consistent loads fall on face centres, which that element
    # does not have)
    "c4s": dict(name="cantilever S2 48x24x24 n=4 mixed", kind="cantilever",
                nel=(48, 24, 24), order=2, nsub=4, nlevels=5, nrhs=1,
                precision="mixed", omega=0.6, pre=1, post=1,
                field="grf", seed=4, family="serendipity"),
    # cubic elements (Sec. 7.5 compares them on the MBB beam with n = 4):
    # the displacement mesh of its quarter model, 48 x 16 x 8 elements
    # (533k DOFs with the 64-node element), point load at the top centre,
    # the finest level smoothed by the multicolour Gauss-Seidel sweep
    "c6": dict(name="mbb L3 48x16x8 n=4 mixed", kind="mbb",
               nel=(48, 16, 8), order=3, nsub=4, nlevels=4, nrhs=1,
               precision="mixed", omega=0.6, pre=1, post=1,
               field="grf", seed=6, smoother="gauss-seidel"),
    "c6s": dict(name="mbb S3 48x16x8 n=4 mixed", kind="mbb",
                nel=(48, 16, 8), order=3, nsub=4, nlevels=4, nrhs=1,
                precision="mixed", omega=0.6, pre=1, post=1,
                field="grf", seed=6, family="serendipity", smoother="gauss-seidel"),
}

SERVE_MESHES = [(32, 16, 16), (48, 24, 24), (64, 32, 32), (96, 48, 48), (128, 64, 64)]
# Poisson arrival rate of the served mix (requests per second), frozen at
# 0.8 x the closed-loop capacity of the FP64 path on one MI355X (24.0
# solves/s with every request queued at once, 5 solves per request); both
# precisions are served at this rate.
SERVE_RATE = {"fp64": 3.84, "mixed": 3.84}
SERVE_NSUB = [1, 2, 4]
SERVE_KINDS = ["cantilever", "mbb", "torsion"]


def config(name):
    return dict(CONFIGS[name])


def densities(cfg, seed=None):
    """Density field of a workload, C-order (nz*n, ny*n, nx*n)."""
    n = cfg["nsub"]
    nx, ny, nz = cfg["nel"]
    shape = (nz * n, ny * n, nx * n)
    s = cfg["seed"] if seed is None else seed
    if cfg["field"] == "uniform":
        return uniform_field(shape, s, 0.05, 1.0)
    return gaussian_random_field(shape, s, corr=6.0, rho_min=1e-3, volfrac=0.3)


def problem(cfg):
    nx, ny, nz = cfg["nel"]
    return make_problem(cfg["kind"], nx, ny, nz, cfg["order"], cfg["nrhs"])


def coarsest_levels(nel, order=1, max_coarse_dof=700):
    """Number of multigrid levels for a served mesh: halve while every
    element count stays even and the coarse lattice is still large."""
    nx, ny, nz = nel
    levels = 2 if order == 2 else 1
    cx, cy, cz = nx, ny, nz
    while cx % 2 == 0 and cy % 2 == 0 and cz % 2 == 0 and \
            3 * (cx + 1) * (cy + 1) * (cz + 1) > max_coarse_dof:
        cx, cy, cz = cx // 2, cy // 2, cz // 2
        levels += 1
    return levels


def serve_requests(n=256, seed=5, rate=None, solves_per_session=5):
    """The served mix: Poisson arrivals (times in seconds for `rate` requests
    per second; `None` leaves arrival times unset), uniform choices of
    structure, mesh, density subdivision and 1-4 load cases."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for r in range(n):
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        kind = SERVE_KINDS[rng.integers(len(SERVE_KINDS))]
        mesh = SERVE_MESHES[rng.integers(len(SERVE_MESHES))]
        nsub = SERVE_NSUB[rng.integers(len(SERVE_NSUB))]
        nrhs = int(rng.integers(1, 5))
        out.append(dict(id=r, arrival=t if rate is not None else None, kind=kind,
                        nel=mesh, nsub=nsub, nrhs=nrhs, order=1,
                        nlevels=coarsest_levels(mesh),
                        seed=50000 + r,
                        perturb_seeds=[60000 + 10 * r + s for s in range(1, solves_per_session)]))
    return out


def serve_base_fields(reqs):
    """One seeded Gaussian random field per (mesh, n) cell of the mix, seeds
    70000, 70001, ... in order of the cells' first request."""
    bases = {}
    for q in reqs:
        key = (q["nel"], q["nsub"])
        if key not in bases:
            nx, ny, nz = q["nel"]
            m = q["nsub"]
            bases[key] = gaussian_random_field((nz * m, ny * m, nx * m), 70000 + len(bases))
    return bases


def serve_densities(bases, req, mask, f, k):
    """Densities of solve k of a request's session: its cell's base field
    perturbed with the request's k-th seed, then solid (1) in every element
    touching one of its supports or loads.  Without the solid layers some
    MBB requests under the top-face pressure hold their load in void: |u|
    reaches 1e7-1e9 and no FP64 solve gets ||f - K u|| below 1e-8 ||f||
    (rounding in K u alone is about eps |K| |u|)."""
    seed = req["seed"] if k == 0 else req["perturb_seeds"][k - 1]
    rho = perturb(bases[(req["nel"], req["nsub"])], seed)
    return solid_at_supports_and_loads(rho, mask, f, req["nel"], req["nsub"])


__all__ = ["MATERIAL", "CONFIGS", "SERVE_RATE", "config", "densities", "problem", "serve_requests",
           "serve_base_fields", "serve_densities", "coarsest_levels", "perturb"]
