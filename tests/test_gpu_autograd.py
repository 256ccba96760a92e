"""Compliance and its gradient through torch.autograd (the device adjoint
kernel) against the oracle's direct solve and against central finite
differences of the compliance."""

import numpy as np
import pytest

from helpers import Case, need_gpu, rel

pytestmark = pytest.mark.gpu


def _compliance_energy(p, f):
    """c~ = f.u + u.(f - K u) for the current solution: equal to f.u at the
    exact solution and accurate to second order in the solve error (the
    energy identity), so that a central difference at h = 1e-6 is limited by
    rounding, not by the solver tolerance."""
    u = p.displacement()
    Ku = p.apply(0, u)
    return float(np.sum(f * u) + np.sum(u * (f - Ku)))


@pytest.mark.parametrize("nsub,precision", [(1, "fp64"), (2, "fp64"), (4, "mixed")])
def test_gradient_matches_oracle(nsub, precision):
    need_gpu()
    import torch
    from paper_2311_05595_amd import autograd
    # a uniform field: on rough fields with densities down to 1e-3 and two
    # levels, 1e-10 is below the attainable accuracy (the oracle's own MG-CG
    # stagnates near 4e-9 on such a case)
    c = Case("cantilever", (8, 4, 4), 1, nsub, 2, 1, field="uniform", seed=31, precision=precision)
    p = c.problem()
    rho = torch.tensor(c.rho, dtype=torch.float64, device="cuda", requires_grad=True)
    comp = autograd.compliance(rho, p, rtol=1e-10, warm_start=False)
    (2.0 * comp).backward()
    g = rho.grad.detach().cpu().numpy().ravel()
    ud = c.direct()
    cref = c.compliance(ud).sum()
    assert abs(comp.item() - cref) <= 1e-9 * cref
    assert rel(g, 2.0 * c.sensitivity(ud)) <= 1e-8
    assert np.all(g <= 0.0)
    p.close()


@pytest.mark.parametrize("seed", range(32))
def test_gradient_matches_central_differences(seed):
    """Directional central difference along a seeded Rademacher direction on
    a seeded multiresolution density field (4^3 sub-elements per element),
    h = 1e-6.  The quotient's error is the rounding of the two compliance
    values divided by 2h: summed in FP64 over ~10^4 terms, c carries a
    relative rounding of ~1e-14 (the same quotient from the oracle's direct
    solves shows 1-2e-14 c), hence the bound 1e-6 |dc.v| + 5e-14 c / h."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import autograd
    nel, nsub = (8, 4, 4), 4
    c = Case("cantilever", nel, 1, nsub, 2, 1, field="uniform", seed=3000 + seed)
    p = c.problem()
    rho0 = torch.tensor(c.rho, dtype=torch.float64, device="cuda", requires_grad=True)
    comp = autograd.compliance(rho0, p, rtol=1e-12, warm_start=False)
    comp.backward()
    g = rho0.grad.detach().cpu().numpy().ravel()
    v = np.random.default_rng(3100 + seed).choice([-1.0, 1.0], size=c.rho.size)
    h = 1e-6
    f = c.f
    vals = []
    for s in (1.0, -1.0):
        r = torch.tensor(c.rho.ravel() + s * h * v, dtype=torch.float64, device="cuda")
        p.set_densities(r)
        info = p.solve(rtol=1e-12, maxit=3000, warm_start=True)
        assert info["status"] == 0
        vals.append(_compliance_energy(p, f))
    fd = (vals[0] - vals[1]) / (2 * h)
    an = float(g @ v)
    assert abs(fd - an) <= 1e-6 * abs(an) + 5e-14 * abs(comp.item()) / h
    p.close()


def test_gradient_central_differences_64x32x32_n4_mixed():
    """The multiresolution workload at its full size (64x32x32 elements, 4^3
    densities each, 4.2M densities, mixed precision): 32 seeded density
    fields (the workload's random field with seeded +-0.05 perturbations),
    each with a directional central difference (h = 1e-6) along a seeded
    Rademacher direction against dc.v from the adjoint kernel.  Compliance
    values from the energy-corrected c~ (second order in the solve error);
    bound as above with the rounding of c over ~2e5 terms."""
    need_gpu()
    import torch
    import workloads as W
    from workloads import configs as CF
    from paper_2311_05595_amd import api, autograd
    cfg = CF.config("c3")
    mask, f = CF.problem(cfg)
    base = CF.densities(cfg)
    p = api.Problem(cfg["nel"], mask, f, order=1, nsub=cfg["nsub"], nlevels=cfg["nlevels"],
                    precision=cfg["precision"], omega=cfg["omega"])
    h = 1e-6
    worst = 0.0
    for k in range(32):
        rho = W.perturb(base, 3000 + k)
        print(f"[fd c3] field {k}", flush=True)
        t = torch.tensor(rho.ravel(), dtype=torch.float64, device="cuda", requires_grad=True)
        comp = autograd.compliance(t, p, rtol=1e-9, maxit=3000, warm_start=False)
        comp.backward()
        g = t.grad.detach().cpu().numpy()
        v = np.random.default_rng(3100 + k).choice([-1.0, 1.0], size=rho.size)
        # densities within h of a bound (the field is clipped to [1e-3, 1])
        # do not move: both perturbed fields stay admissible
        v[(rho.ravel() > 1.0 - h) | (rho.ravel() < h)] = 0.0
        vals = []
        for s in (1.0, -1.0):
            r = torch.tensor(rho.ravel() + s * h * v, dtype=torch.float64, device="cuda")
            p.set_densities(r)
            info = p.solve(rtol=1e-9, maxit=3000, warm_start=True)
            assert info["status"] == 0
            vals.append(_compliance_energy(p, f))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(g @ v)
        bound = 1e-6 * abs(an) + 2e-13 * abs(comp.item()) / h
        worst = max(worst, abs(fd - an) / bound)
        assert abs(fd - an) <= bound, (k, fd, an)
    print(f"[fd c3] worst |fd - dc.v| / bound = {worst:.3f}", flush=True)
    p.close()
