"""Host checks of the seeded input generators (no GPU, no solver)."""

import numpy as np

import workloads as W
from workloads import configs as CF


def test_solid_layers_cover_supports_and_loads():
    nel, nsub = (6, 4, 2), 2
    for kind in ("cantilever", "mbb", "torsion"):
        mask, f = W.make_problem(kind, *nel, 1, 4)
        rho = W.gaussian_random_field((nel[2] * nsub, nel[1] * nsub, nel[0] * nsub), 7)
        out = W.solid_at_supports_and_loads(rho, mask, f, nel, nsub)
        nx, ny, nz = nel
        touched = (mask.reshape(-1, 3) != 0).any(1) | (f != 0).reshape(f.shape[0], -1, 3).any((0, 2))
        touched = touched.reshape(nz + 1, ny + 1, nx + 1)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    block = out[k * nsub:(k + 1) * nsub, j * nsub:(j + 1) * nsub,
                                i * nsub:(i + 1) * nsub]
                    orig = rho[k * nsub:(k + 1) * nsub, j * nsub:(j + 1) * nsub,
                               i * nsub:(i + 1) * nsub]
                    if touched[k:k + 2, j:j + 2, i:i + 2].any():
                        assert np.all(block == 1.0), (kind, i, j, k)
                    else:
                        assert np.array_equal(block, orig), (kind, i, j, k)
        assert not np.shares_memory(out, rho)


def test_served_mix_is_seeded_and_in_range():
    reqs = CF.serve_requests(12, seed=5, rate=2.0)
    again = CF.serve_requests(12, seed=5, rate=2.0)
    assert [q["nel"] for q in reqs] == [q["nel"] for q in again]
    assert all(np.diff([q["arrival"] for q in reqs]) > 0)
    small = [q for q in reqs if q["nel"] == (32, 16, 16)] or [dict(reqs[0], nel=(32, 16, 16))]
    q = small[0]
    bases = CF.serve_base_fields([q])
    mask, f = W.make_problem(q["kind"], *q["nel"], 1, q["nrhs"])
    a = CF.serve_densities(bases, q, mask, f, 1)
    b = CF.serve_densities(bases, q, mask, f, 1)
    assert np.array_equal(a, b)
    assert a.min() >= 1e-3 and a.max() == 1.0
    assert not np.array_equal(a, CF.serve_densities(bases, q, mask, f, 2))
