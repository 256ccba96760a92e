"""Continuous batching: requests of different sizes, load-case counts and
precisions admitted by HBM budget, overlapping on the device; every result
must equal the same solve run alone, and the oracle's direct solve."""

import numpy as np
import pytest

from helpers import need_gpu, rel

pytestmark = pytest.mark.gpu

# kind, elements, order, n, levels, load cases, precision
SPECS = [
    ("cantilever", (16, 8, 8), 1, 1, 3, 1, "fp64"),
    ("mbb", (8, 4, 4), 1, 2, 2, 2, "mixed"),
    ("torsion", (12, 6, 6), 1, 1, 2, 3, "fp64"),
    ("cantilever", (8, 4, 4), 2, 1, 2, 1, "fp64"),
    ("cantilever", (16, 8, 8), 1, 1, 3, 4, "mixed"),
    ("mbb", (24, 12, 12), 1, 1, 3, 1, "mixed"),
]


def _problem(spec):
    import workloads as W
    from paper_2311_05595_amd import api
    kind, nel, order, nsub, nlev, nrhs, prec = spec
    mask, f = W.make_problem(kind, *nel, order, nrhs)
    return api.Problem(nel, mask, f, order=order, nsub=nsub, nlevels=nlev, precision=prec)


def _fields(spec, seed):
    import workloads as W
    kind, nel, order, nsub, nlev, nrhs, prec = spec
    shape = (nel[2] * nsub, nel[1] * nsub, nel[0] * nsub)
    base = W.gaussian_random_field(shape, seed, corr=3.0)
    return [base, W.perturb(base, seed + 1000)]  # a session: cold solve, then a warm re-solve


def _oracle(spec, rho):
    """The oracle's direct solve of one request: u per load case and c."""
    import workloads as W
    from oracle import assemble, fem, solve
    kind, nel, order, nsub, nlev, nrhs, prec = spec
    mask, f = W.make_problem(kind, *nel, order, nrhs)
    K = assemble.stiffness(rho, nel, order, nsub, fem.sub_element_matrices(order, nsub),
                           E0=1.0, Emin=1e-9, penal=3.0)
    u = solve.solve_direct(K, mask, f)
    return u, solve.compliance(f, u)


def test_alone_equals_mix_and_budget():
    need_gpu()
    from paper_2311_05595_amd import api
    rtol = 1e-10
    # alone: each session on its own, one after the other
    alone = []
    for k, spec in enumerate(SPECS):
        p = _problem(spec)
        us = []
        for j, rho in enumerate(_fields(spec, 50 + k)):
            p.set_densities(rho)
            info = p.solve(rtol=rtol, maxit=3000, warm_start=j > 0)
            assert info["status"] == 0
            us.append(p.displacement().copy())
        alone.append(us)
        p.close()
    # mixed: all sessions submitted at once to a server whose budget holds
    # only some of them, so requests queue and are admitted as memory frees
    probs = [_problem(s) for s in SPECS]
    sizes = [p.device_bytes() for p in probs]
    budget = int(max(sizes) + 0.5 * sum(sorted(sizes)[:-1]))
    srv = api.Server(budget, max_slots=3)
    fields = [_fields(s, 50 + k) for k, s in enumerate(SPECS)]
    tickets = {}
    for k, p in enumerate(probs):
        tickets[srv.submit(p, fields[k][0], rtol=rtol, maxit=3000, warm_start=False)] = (k, 0)
    results, comp, lat = {}, {}, []
    max_active, saw_queue = 0, False
    guard = 0
    while tickets:
        active, queued = srv.step()
        max_active = max(max_active, active)
        saw_queue = saw_queue or queued > 0
        assert srv.resident_bytes() <= budget
        for t in list(tickets):
            out = srv.poll(t)
            if out is None:
                continue
            k, j = tickets.pop(t)
            st, info, ms = out
            assert st == 0, (k, j, st)
            lat.append(ms)
            results[(k, j)] = probs[k].displacement().copy()
            comp[(k, j)] = probs[k].compliance_sensitivity(want_dc=False)[0]
            if j == 0:  # the session's warm-started second solve
                tickets[srv.submit(probs[k], fields[k][1], rtol=rtol, maxit=3000,
                                   warm_start=True)] = (k, 1)
            else:
                srv.release(probs[k])
        guard += 1
        assert guard < 200000
    assert max_active >= 2 and saw_queue
    for k in range(len(SPECS)):
        for j in range(2):
            assert rel(results[(k, j)], alone[k][j]) <= 1e-12, (SPECS[k], j)
            # and the oracle: u within 1e-8, c within 1e-9, per load case
            u_ref, c_ref = _oracle(SPECS[k], fields[k][j])
            for lc in range(SPECS[k][5]):
                assert rel(results[(k, j)][lc], u_ref[lc]) <= 1e-8, (SPECS[k], j, lc)
                assert abs(comp[(k, j)][lc] - c_ref[lc]) <= 1e-9 * abs(c_ref[lc]), (SPECS[k], j)
    lat = np.sort(lat)
    assert lat[0] > 0.0 and np.percentile(lat, 99) >= np.percentile(lat, 50)
    srv.close()
    for p in probs:
        p.close()


def test_budget_rejects_oversized_request():
    need_gpu()
    from paper_2311_05595_amd import api
    from paper_2311_05595_amd._abi import MGCGError, MGCG_EBUDGET
    spec = SPECS[0]
    p = _problem(spec)
    srv = api.Server(p.device_bytes() // 2, max_slots=2)
    with pytest.raises(MGCGError) as e:
        srv.submit(p, _fields(spec, 1)[0])
    assert e.value.code == MGCG_EBUDGET
    srv.close()
    p.close()


def test_device_submit_equals_host_submit():
    """Densities submitted from device memory (copied on the device, in order
    after torch's stream) give the same solve as host densities."""
    need_gpu()
    import torch
    from paper_2311_05595_amd import api
    spec = SPECS[1]
    fields = _fields(spec, 77)
    out = []
    for dev in (False, True):
        p = _problem(spec)
        srv = api.Server(4 * p.device_bytes(), max_slots=2)
        us = []
        for j, rho in enumerate(fields):
            src = torch.tensor(rho.ravel(), dtype=torch.float64, device="cuda") if dev else rho
            t = srv.submit(p, src, rtol=1e-12, maxit=3000, warm_start=j > 0)
            if dev:
                src.fill_(-1.0)  # the caller may reuse its buffer once submit returns
            while True:
                srv.step()
                r = srv.poll(t)
                if r is not None:
                    break
            assert r[0] == 0
            us.append(p.displacement().copy())
        srv.release(p)
        srv.close()
        p.close()
        out.append(us)
    for j in range(2):
        assert rel(out[1][j], out[0][j]) <= 1e-14
    u_ref, _ = _oracle(spec, fields[1])
    assert rel(out[1][1], u_ref) <= 1e-8


def test_destroy_with_running_request_returns():
    """Destroying a server while a request is mid-solve waits only for the
    work already queued, and the problem stays usable."""
    need_gpu()
    from paper_2311_05595_amd import api
    spec = SPECS[5]
    p = _problem(spec)
    rho = _fields(spec, 5)[0]
    srv = api.Server(2 * p.device_bytes(), max_slots=1)
    t = srv.submit(p, rho, rtol=1e-14, maxit=5000, warm_start=False)
    active, _ = srv.step()
    assert active == 1 and srv.poll(t) is None
    srv.close()  # must return although the solve has not converged
    p.set_densities(rho)
    info = p.solve(rtol=1e-10, maxit=3000, warm_start=False)
    assert info["status"] == 0
    p.close()
