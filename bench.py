"""Benchmark of the MGCG hot path on one MI355X.

A step = one SLP-like iteration of the optimisation loop on the
96x48x48 trilinear cantilever (0.69M DOF, 5 multigrid levels, FP64): operator
refresh from a perturbed density field (SIMP moduli, Galerkin coarse
operators, Jacobi data, coarsest inverse), a warm-started MGCG solve to a
1e-8 relative residual, and compliance + sensitivity.  The ten perturbed
fields are generated and uploaded before timing; steps cycle through them.

Prints one JSON line.  Besides the contract's keys:
* `roofline`: the finest-level CG apply (per-launch HIP events on the
  library's stream over the timed steps) against its algorithmic work;
* `accuracy`: FP64 and mixed-precision solves of one field (warm-started as
  in the timed steps, and cold) against the oracle's MG-CG reference run to
  a tight residual: relative errors of u and c, iterations;
* `cpu_baseline`: the oracle's cold solve from that same run (setup + the
  iterations it needed to 1e-8), on one host thread, with the host's CPU;
* `served`: the served mix (the fifth workload) on the FP64 and the mixed
  path, at the frozen Poisson rate and at capacity (`--no-served` skips it).
`--config c1|c3|c4|c4s|c6|c6s` times the other single-GPU workloads the
same way (not the default line; no served legs), `--config c5` the served
mix alone.  `--launch fused` runs each solve as one launch (a workgroup per
load case; small trilinear FP64 workloads such as c1), then without the
per-kernel roofline.
`--copy-probe MIB` only runs the library's plain copy kernel on MIB MiB
(the calibration run for the HBM byte counters) and exits.

`--apply-sweep` times the matrix-free CG apply of the trilinear cantilever
on lattices from 96x48x48 to 224x112x112 elements (FP64 and mixed) and
prints one JSON line with its fraction of the FP64 peak per lattice.

`--projection` times the design-variable projection rho = W x and its
transpose W^T g (Sec. 3.2 eq. (5), Sec. 3.4) on the 64x32x32 mesh with 4^3
density and 2^3 design cells per element, rmin = 1.5, and prints its own
JSON line (kernel rooflines and the oracle's single-entry evaluation timed
on a sample).

`--lp` times the SLP step's LP subproblem (Sec. 4.1) over the 524,288 design
variables of that lattice and prints its own JSON line.

`--threshold` times the density thresholding of Sec. 5 on the 4,194,304
densities of that lattice: the rule based on the density values (the
printed line), the Heaviside projection with Newton's volume-preserving
threshold, the angle condition's cosine and the strategy based on the
gradient of the Lagrangian (in `config`).

`--fixing` times the choice of fixed variables of Sec. 6.1 on that mesh
(4^3 densities, 2^3 design cells per element, the Q2 node lattice).
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks (datasheet): HBM3E 8 TB/s; FP64 vector 78.6 TFLOP/s
# (256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU); FP32 vector 157.3 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that make up the finest-level apply kernel; the committed HBM
# traffic figure is reported only while they are unchanged.
KERNEL_SOURCES = ["k_apply.hip", "kernels.h", "devutil.h", "common.h", "q1table.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mf_q1_apply_cantilever_96x48x48.md")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_05595_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic():
    """HBM bytes per launch of the finest-level apply from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    the summary is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mib):
    import torch
    import workloads as W
    from paper_2311_05595_amd import api
    n = mib * 1024 * 1024
    dev = torch.device("cuda:0")
    a = torch.ones(n // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    mask, f = W.make_problem("cantilever", 4, 2, 2, 1, 1)
    prob = api.Problem((4, 2, 2), mask, f, nlevels=1)
    prob.use_torch_stream()
    for _ in range(5):
        prob.copy_bytes(a.data_ptr(), b.data_ptr(), n)
    torch.cuda.synchronize()
    assert bool((b == 1).all())
    prob.close()
    print(json.dumps({"copy_probe_bytes": n, "launches": 5}), flush=True)


def fine_apply_model(nel, nsub, order, nrhs=1, family="lagrange"):
    """The finest-level operator of a workload and the algorithmic work of one
    CG apply q = A p with it (per launch = all elements and load cases):
    * trilinear, one density per element (matrix-free, unit element matrix
      scaled per element): 24x24 matvec per element = 1152 flop; bytes: read
      p and E, write q.  Bound: FP64 ALU.
    * trilinear with n^3 densities per element (assembled 27-point stencil,
      symmetric half: 14 blocks of 3x3 per node): bytes: the 126 stencil
      coefficients per node, read p, write q.  Bound: HBM.
    * triquadratic (stored symmetric 81x81 element matrices): bytes: the
      3321 distinct coefficients per element, read p, write q.  Bound: HBM.
    * quadratic serendipity (stored symmetric 60x60 element matrices): the
      1830 distinct coefficients per element, read p, write q.  Bound: HBM.
    * tricubic (stored symmetric 192x192 element matrices, or 96x96 for the
      32-node serendipity element): the 18528 (4656) distinct coefficients
      per element, read p, write q.  Bound: HBM."""
    nx, ny, nz = nel
    nelem = nx * ny * nz
    nn = (order * nx + 1) * (order * ny + 1) * (order * nz + 1)
    ndof = 3 * nn
    vec = 8.0 * 2 * ndof * nrhs
    if order == 1 and nsub == 1:
        return dict(bound="alu", flops=1152.0 * nelem * nrhs, bytes=vec + 8.0 * nelem,
                    kernel="finest-level CG apply q = A p, matrix-free trilinear (FP64)",
                    per_unit="1152 flop per element and load case")
    if order == 1:
        return dict(bound="hbm", flops=2.0 * 243 * nn * nrhs, bytes=vec + 8.0 * 126 * nn,
                    kernel="finest-level CG apply q = A p, 27-point stencil (FP64)",
                    per_unit="126 x 8 B of coefficients per node + 48 B of vectors per node "
                             "and load case")
    if order == 3:
        nd = 96 if family == "serendipity" else 192
        kc = nd * (nd + 1) // 2
        what = "serendipity " if family == "serendipity" else ""
        return dict(bound="hbm", flops=2.0 * nd * nd * nelem * nrhs, bytes=vec + 8.0 * kc * nelem,
                    kernel=f"finest-level CG apply q = A p, stored symmetric {nd}x{nd} {what}"
                           "element matrices (FP64)",
                    per_unit=f"{kc} x 8 B of element matrix (distinct entries) per element + 48 B "
                             "of vectors per node and load case")
    if family == "serendipity":
        return dict(bound="hbm", flops=2.0 * 3600 * nelem * nrhs, bytes=vec + 8.0 * 1830 * nelem,
                    kernel="finest-level CG apply q = A p, stored symmetric 60x60 serendipity "
                           "element matrices (FP64)",
                    per_unit="1830 x 8 B of element matrix (distinct entries) per element + 48 B "
                             "of vectors per node and load case")
    return dict(bound="hbm", flops=2.0 * 6561 * nelem * nrhs, bytes=vec + 8.0 * 3321 * nelem,
                kernel="finest-level CG apply q = A p, stored symmetric 81x81 element matrices "
                       "(FP64)",
                per_unit="3321 x 8 B of element matrix (distinct entries) per element + 48 B of "
                         "vectors per node and load case")


def batch_bench(args):
    """Many small problems (the c1 workload's mesh and settings, each with its
    own seeded density field): every step refreshes all of them and solves
    them warm-started to 1e-8, either one after another on the eager path or
    all in one fused launch (mgcg_solve_batch, a workgroup per problem); the
    solves are timed, the refreshes before them are not.  Prints one JSON
    line with both rates; not the default line."""
    import torch
    import workloads as W
    from workloads import configs as CF
    from paper_2311_05595_amd import api
    cfg = CF.config("c1")
    mask, f = CF.problem(cfg)
    n = args.batch
    fields = [[W.perturb(W.uniform_field(cfg["nel"][::-1], 100 + i), 9000 + 31 * i + k)
               for k in range(3)] for i in range(n)]
    probs = [api.Problem(cfg["nel"], mask, f, nlevels=cfg["nlevels"], omega=cfg["omega"])
             for _ in range(n)]
    out = {"metric": "batched small-problem MGCG solves/s at 1e-8 rel. residual",
           "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "config": {"workload": cfg["name"] + f", {n} problems with their own seeded "
                      "densities, warm-started", "problems": n, "steps": args.steps}}
    for mode in args.batch_modes.split(","):
        for p in probs:
            p.set_launch_mode(mode)
        iters = []

        def step(k):
            # the refresh of every problem, then the timed solves
            for i, p in enumerate(probs):
                p.set_densities(fields[i][k % 3].ravel())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "fused":
                infos = api.solve_batch(probs, rtol=1e-8, maxit=2000, warm_start=k > 0)
            else:
                infos = [p.solve(rtol=1e-8, maxit=2000, warm_start=k > 0) for p in probs]
            torch.cuda.synchronize()
            iters.extend(i["iters"][0] for i in infos)
            return time.perf_counter() - t0
        step(0)
        iters.clear()
        el = sum(step(k) for k in range(1, args.steps + 1))
        out[mode] = {"solves_s": round(n * args.steps / el, 2), "ms_per_step": round(el / args.steps * 1e3, 3),
                     "pcg_iters_mean": round(float(np.mean(iters)), 2)}
    out["value"] = out.get("fused", out.get("eager", {})).get("solves_s")
    for p in probs:
        p.close()
    print(json.dumps(out), flush=True)


def apply_sweep(args):
    """The finest-level matrix-free CG apply of the trilinear cantilever on
    growing lattices (single density per element, seeded uniform densities in
    [0.1, 1]): 60 PCG iterations per lattice and precision, the apply's mean
    duration from HIP events on the library's stream, against the FP64 peak.
    Prints one JSON line; not the default line."""
    import torch
    import workloads as W
    from paper_2311_05595_amd import api
    rows = []
    for nel, nl in [((96, 48, 48), 5), ((128, 64, 64), 6), ((160, 80, 80), 5),
                    ((192, 96, 96), 6), ((224, 112, 112), 5)]:
        for prec in ("fp64", "mixed"):
            mask, f = W.make_problem("cantilever", *nel, 1, 1)
            p = api.Problem(nel, mask, f, order=1, nsub=1, nlevels=nl, precision=prec)
            p.use_torch_stream()
            rho = np.random.default_rng(0).uniform(0.1, 1.0, nel[::-1]).ravel()
            p.set_densities(torch.tensor(rho, dtype=torch.float64, device="cuda"))
            p.solve(rtol=1e-30, maxit=10, warm_start=False, allow_notconv=True)
            torch.cuda.synchronize()
            p.set_kernel_timing(0, True)
            t0 = time.perf_counter()
            p.solve(rtol=1e-30, maxit=60, warm_start=False, allow_notconv=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ms, n = p.kernel_timing(0)
            p.set_kernel_timing(0, False)
            p.close()
            m = fine_apply_model(nel, 1, 1)
            avg = ms / n * 1e-3
            tf = m["flops"] / avg / 1e12
            rows.append({"nel": list(nel), "precision": prec, "dof": 3 * (nel[0] + 1) * (nel[1] + 1) * (nel[2] + 1),
                         "apply_us": round(avg * 1e6, 2), "TFLOP_s": round(tf, 2),
                         "frac": round(tf / PEAK_FP64_TFLOPS, 3), "us_per_iteration": round(el / 60 * 1e6, 1)})
            print(f"[sweep] {nel} {prec}: {avg * 1e6:.2f} us, frac {tf / PEAK_FP64_TFLOPS:.3f}", flush=True)
    print(json.dumps({"metric": "finest-level CG apply, matrix-free trilinear, vs lattice size",
                      "kernel": "finest-level CG apply q = A p (FP64)", "per_unit": "1152 flop per element",
                      "peak_TFLOP_s": PEAK_FP64_TFLOPS, "rows": rows}), flush=True)


def host_info():
    """The host the oracle runs on: logical CPUs and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model}


def oracle_reference(cfg, rho, rtol_ref=1e-12, max_iters=400, budget_s=60.0):
    """The oracle on one density field of the workload, on one host thread:
    assemble K, build the Galerkin hierarchy and run its MG-preconditioned CG
    (Algorithm 1, the same stopping rule) from zero to rel. residual
    `rtol_ref` (or the iteration / time cap).  Returns the reference
    solution u*, c* = f.u*, and the timings that give the CPU baseline: the
    setup time, the time per CG iteration and the iteration at which the
    residual first fell below 1e-8 (a cold solve)."""
    from threadpoolctl import threadpool_limits
    from oracle import assemble, fem, multigrid
    from workloads import configs as CF
    mask, f = CF.problem(cfg)
    nel, order, nsub = cfg["nel"], cfg["order"], cfg["nsub"]
    family = cfg.get("family", "lagrange")
    if family == "serendipity":
        mask = np.maximum(mask, fem.serendipity_dof_mask(nel, order))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        Ks = fem.sub_element_matrices(order, nsub, family=family)
        K = assemble.stiffness(rho, nel, order, nsub, Ks)
        A0 = assemble.level_operator(K, mask)
        H = multigrid.Hierarchy(A0, mask, assemble.node_dims(nel, order), cfg["nlevels"], order0=order)
        weights = multigrid.smoother_weights(H, cfg["omega"])
        t_setup = time.perf_counter() - t0
        us, it8, its, res = [], None, 0, 0.0
        t1 = time.perf_counter()
        for lc in range(f.shape[0]):
            b = f[lc].copy()
            b[mask.astype(bool)] = 0.0
            x = np.zeros_like(b)
            r = b.copy()
            nf = np.linalg.norm(b)
            z = multigrid.vcycle(H, r, weights=weights)
            p = z.copy()
            rz = r @ z
            it = 0
            while it < max_iters and time.perf_counter() - t1 < budget_s:
                q = H.A[0] @ p
                a = rz / (p @ q)
                x += a * p
                r -= a * q
                it += 1
                rel = np.linalg.norm(r) / nf
                if lc == 0 and it8 is None and rel <= 1e-8:
                    it8 = it
                if rel <= rtol_ref:
                    r = b - H.A[0] @ x  # the true residual decides
                    if np.linalg.norm(r) / nf <= rtol_ref:
                        break
                z = multigrid.vcycle(H, r, weights=weights)
                rzn = r @ z
                p = z + (rzn / rz) * p
                rz = rzn
            its += it
            res = max(res, np.linalg.norm(b - H.A[0] @ x) / nf)
            us.append(x)
        t_iter = (time.perf_counter() - t1) / max(its, 1)
    u = np.stack(us)
    c = float(np.einsum("ld,ld->", f, u))
    return dict(u=u, c=c, t_setup=t_setup, t_iter=t_iter, iters=its, it8=it8, rel_res=res,
                rtol=rtol_ref)


def cpu_baseline_from(ref, cfg):
    """The oracle's cold solve to 1e-8 on one host thread (setup + the CG
    iterations it needed), from the reference run."""
    need = ref["it8"] if ref["it8"] is not None else float("nan")
    t_solve = (ref["t_setup"] + need * ref["t_iter"]) * cfg["nrhs"]
    out = dict(value=1.0 / t_solve, unit="solves/s", cores=1, kind="oracle",
               sample=(f"oracle (NumPy/SciPy FP64, 1 thread; BLAS limited to 1) on one density "
                       f"field of the workload ({cfg['name']}), cold start: assembly + Galerkin "
                       f"hierarchy {ref['t_setup']:.1f} s, {need} MG-preconditioned CG "
                       f"iterations to rel. residual 1e-8 at {ref['t_iter']:.3f} s each "
                       f"(timed inside a run to {ref['rtol']:.0e}, {ref['iters']} iterations); "
                       f"x{cfg['nrhs']} load cases = {t_solve:.1f} s per solve.  The GPU steps "
                       f"are warm-started; the GPU's cold solve of the same field is "
                       f"accuracy.fp64.cold"))
    out.update(host_info())
    out["threads"] = 1
    return out


def run(args):
    import torch
    import workloads as W
    from workloads import configs as CF
    from paper_2311_05595_amd import api

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
        sys.exit(2)
    cfg = CF.config(args.config)
    mask, f = CF.problem(cfg)
    base = CF.densities(cfg)
    seeds = cfg.get("perturb_seeds") or list(range(9001, 9011))
    fields = [W.perturb(base, s) for s in seeds]
    dev = torch.device("cuda:0")
    dfields = [torch.tensor(r.ravel(), dtype=torch.float64, device=dev) for r in fields]
    smoother = args.smoother or cfg.get("smoother", "jacobi")
    prob = api.Problem(cfg["nel"], mask, f, order=cfg["order"], nsub=cfg["nsub"],
                       nlevels=cfg["nlevels"], precision=args.precision or cfg["precision"],
                       omega=cfg["omega"], pre=cfg["pre"], post=cfg["post"],
                       family=cfg.get("family", "lagrange"), smoother=smoother)
    prob.use_torch_stream()
    prob.set_launch_mode(args.launch)
    dc = torch.empty(prob.nrho, dtype=torch.float64, device=dev)
    free = int((mask == 0).sum()) * prob.nrhs
    # cold solve of the base design (the optimisation's first iteration)
    prob.set_densities(torch.tensor(base.ravel(), dtype=torch.float64, device=dev))
    prob.solve(rtol=args.rtol, maxit=args.maxit, warm_start=False)

    def step(k):
        prob.set_densities(dfields[k % len(dfields)])
        info = prob.solve(rtol=args.rtol, maxit=args.maxit, warm_start=True)
        c, _ = prob.compliance_sensitivity(dc_out=dc)
        return info, c

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    # (kernel timing launches eagerly: a fused solve is timed whole)
    timed = args.launch != "fused"
    prob.set_kernel_timing(0, timed)
    lat, iters, statuses = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        info, c = step(args.warmup + k)
        lat.append((time.perf_counter() - ts) * 1e3)
        iters.append(max(info["iters"][:prob.nrhs]))
        statuses.append(info["status"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, kn = prob.kernel_timing(0)
    prob.set_kernel_timing(0, False)

    m = fine_apply_model(cfg["nel"], cfg["nsub"], cfg["order"], prob.nrhs,
                         cfg.get("family", "lagrange"))
    avg_s = (kms / kn) * 1e-3 if kn else float("nan")
    if m["bound"] == "alu":
        achieved, peak, unit = m["flops"] / avg_s / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
    else:
        achieved, peak, unit = m["bytes"] / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    traffic = committed_traffic() if cfg["name"] == CF.config("c2")["name"] else None
    roofline = None if not timed else {
                "bound": m["bound"], "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": m["kernel"], "per_unit": m["per_unit"],
                "avg_us": round(avg_s * 1e6, 3), "launches": kn,
                "alg_flop_per_launch": m["flops"], "alg_bytes_per_launch": m["bytes"],
                "alg_GBs": round(m["bytes"] / avg_s / 1e9, 1),
                "alg_TFLOPs": round(m["flops"] / avg_s / 1e12, 3)}
    lat_s = sorted(lat)
    out = {
        "metric": "MGCG solves/s and DOF·CG-iter/s at 1e-8 rel. residual; p50/p99 solve latency",
        "value": round(args.steps / elapsed, 3),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if (args.precision or cfg["precision"]) == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + ", warm-started over 10 seeded +-0.05 density "
                   "perturbations; step = refresh + solve + compliance/sensitivity",
                   "nel": list(cfg["nel"]), "free_dof": free, "levels": cfg["nlevels"],
                   "rtol": args.rtol, "smoother": smoother, "launch": args.launch},
        "dof_cg_iter_per_s": round(free * sum(iters) / elapsed, 1),
        "pcg_iters_mean": round(float(np.mean(iters)), 2),
        "p50_ms": round(lat_s[len(lat_s) // 2], 3),
        "p99_ms": round(lat_s[min(len(lat_s) - 1, int(math.ceil(0.99 * len(lat_s))) - 1)], 3),
        "statuses": sorted(set(statuses)),
        "not_converged": sum(1 for s in statuses if s != 0),
        "roofline": roofline,
    }
    if not args.no_cpu:
        log("oracle reference solve on the host ...")
        ref = oracle_reference(cfg, fields[0], budget_s=args.cpu_budget)
        out["accuracy"] = accuracy_legs(args, cfg, mask, f, base, fields[0], prob, ref)
        out["cpu_baseline"] = cpu_baseline_from(ref, cfg)
    if not args.no_served and args.config == "c2":
        # the served mix on both paths: Poisson arrivals at the frozen rate
        # (throughput = offered load; latency differs), then every request
        # queued at once (capacity: solves/s differ)
        out["served"] = {}
        for leg in ("fp64", "mixed"):
            entry = {}
            for mode, rate, nreq in (("poisson", 0.0, args.requests),
                                     ("capacity", 1000.0, args.requests // 2)):
                log(f"served mix, {leg}, {mode} ...")
                sv = served_mix(args, leg, rate=rate, requests=nreq)
                entry[mode] = {"solves_s": sv["value"], "p50_ms": sv["p50_ms"],
                               "p99_ms": sv["p99_ms"], "dof_cg_iter_per_s": sv["dof_cg_iter_per_s"],
                               "not_converged": sv["not_converged"], "solves": sv["steps"],
                               "elapsed_s": sv["elapsed_s"], "rate": sv["rate"]}
            out["served"][leg] = entry
        out["served"]["workload"] = (f"served mix: {args.requests} requests (cantilever / MBB / "
                                     f"torsion; meshes 32x16x16 ... 128x64x64; n in 1,2,4; 1-4 "
                                     f"load cases), {args.session_solves} warm-started solves per "
                                     f"session, HBM budget {args.budget_gb} GB, {args.slots} "
                                     f"slots; poisson: arrivals at the frozen rate; capacity: "
                                     f"the first {args.requests // 2} requests queued at once")
    print(json.dumps(out), flush=True)


def accuracy_legs(args, cfg, mask, f, base, rho, prob, ref):
    """FP64 and mixed-precision solves of one field of the workload against
    the oracle's reference solution u* (its MG-CG run to a tight residual):
    the warm-started solve as in the timed steps (from the solution of the
    previous design), then a cold solve of the same field."""
    import torch
    from paper_2311_05595_amd import api
    dev = torch.device("cuda:0")
    bench_prec = args.precision or cfg["precision"]
    ustar, cstar = ref["u"], ref["c"]
    out = {"reference": {"solver": "oracle MG-preconditioned CG (FP64, 1 thread)",
                         "rel_res": float(f"{ref['rel_res']:.3g}"), "iters": ref["iters"],
                         "iters_to_1e-8": ref["it8"]}}
    drho = torch.tensor(rho.ravel(), dtype=torch.float64, device=dev)
    for leg in ("fp64", "mixed"):
        if leg == bench_prec:
            q = prob
        else:
            q = api.Problem(cfg["nel"], mask, f, order=cfg["order"], nsub=cfg["nsub"],
                            nlevels=cfg["nlevels"], precision=leg, omega=cfg["omega"],
                            pre=cfg["pre"], post=cfg["post"], family=cfg.get("family", "lagrange"),
                            smoother=args.smoother or cfg.get("smoother", "jacobi"))
            q.use_torch_stream()
            q.set_densities(torch.tensor(base.ravel(), dtype=torch.float64, device=dev))
            q.solve(rtol=args.rtol, maxit=args.maxit, warm_start=False)
        q.set_densities(drho)
        iw = q.solve(rtol=args.rtol, maxit=args.maxit, warm_start=True)
        uw = q.displacement()
        cw = float(q.compliance_sensitivity(want_dc=False)[0][q.nrhs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ic = q.solve(rtol=args.rtol, maxit=args.maxit, warm_start=False)
        torch.cuda.synchronize()
        t_cold = time.perf_counter() - t0
        uc = q.displacement()
        cc = float(q.compliance_sensitivity(want_dc=False)[0][q.nrhs])
        nu = np.linalg.norm(ustar)
        out[leg] = {
            "rtol": args.rtol,
            "warm": {"u_rel_err": float(f"{np.linalg.norm(uw - ustar) / nu:.3g}"),
                     "c_rel_err": float(f"{abs(cw - cstar) / abs(cstar):.3g}"),
                     "iters": max(iw["iters"][:q.nrhs]),
                     "rel_res": float(f"{max(iw['rel_res'][:q.nrhs]):.3g}")},
            "cold": {"u_rel_err": float(f"{np.linalg.norm(uc - ustar) / nu:.3g}"),
                     "c_rel_err": float(f"{abs(cc - cstar) / abs(cstar):.3g}"),
                     "iters": max(ic["iters"][:q.nrhs]),
                     "rel_res": float(f"{max(ic['rel_res'][:q.nrhs]):.3g}"),
                     "solve_ms": round(t_cold * 1e3, 3)},
        }
        if q is not prob:
            q.close()
    return out


def run_served(args):
    print(json.dumps(served_mix(args, args.precision or "mixed")), flush=True)


def served_mix(args, prec, rate=None, requests=None):
    """The served mix: sessions of warm-started solves over requests of
    different meshes, density subdivisions, structures and load-case counts,
    arriving as a Poisson process and admitted by an HBM budget.

    The densities of each solve are the client's: a pool of host threads
    makes them (perturbation of the cell's base field, solid layers at the
    request's supports and loads) while the server loop runs, one solve
    ahead per session.  A solve's latency runs from its submission, which
    copies the densities, to the server step that sees it finish."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import workloads as W
    from workloads import configs as CF
    from paper_2311_05595_amd import api
    n = requests or args.requests
    if rate is None:
        rate = args.rate
    rate = rate if rate else CF.SERVE_RATE[prec]
    reqs = CF.serve_requests(n, seed=5, rate=rate, solves_per_session=args.session_solves)
    bases = CF.serve_base_fields(reqs)
    log(f"served mix: {n} requests x {args.session_solves} solves, {len(bases)} base fields, "
        f"rate {rate:.2f} requests/s, budget {args.budget_gb} GB, {prec}")
    pool = ThreadPoolExecutor(max_workers=8)

    def densities(q, mask, f, k):
        return CF.serve_densities(bases, q, mask, f, k)

    srv = api.Server(int(args.budget_gb * 2**30), max_slots=args.slots)
    torch.cuda.synchronize()
    pending = list(reqs)
    tickets = {}    # ticket -> (request index, solve index)
    probs = {}      # request index -> (problem, request, mask, f)
    ready = {}      # request index -> (solve index, future of its densities)
    busy = set()    # requests with a solve submitted and not yet finished
    lat, statuses, failed = [], [], []
    dof_iters = 0
    t0 = time.perf_counter()
    done_solves = 0
    next_report = 15.0
    while pending or tickets or ready:
        now = time.perf_counter() - t0
        if now >= next_report:
            log(f"  t={now:.0f}s: {done_solves} solves done, {len(tickets)} in flight, "
                f"{len(ready)} being prepared, {len(pending)} requests not yet arrived")
            next_report += 15.0
        while pending and pending[0]["arrival"] <= now:
            q = pending.pop(0)
            mask, f = W.make_problem(q["kind"], *q["nel"], 1, q["nrhs"])
            p = api.Problem(q["nel"], mask, f, order=1, nsub=q["nsub"], nlevels=q["nlevels"],
                            precision=prec)
            probs[q["id"]] = (p, q, mask, f)
            ready[q["id"]] = (0, pool.submit(densities, q, mask, f, 0))
        for qid in [i for i, (_, fut) in ready.items() if fut.done() and i not in busy]:
            k, fut = ready.pop(qid)
            p, q, mask, f = probs[qid]
            tickets[srv.submit(p, fut.result(), rtol=1e-8, maxit=2000, warm_start=k > 0)] = (qid, k)
            busy.add(qid)
            if k + 1 < args.session_solves:       # prepare the session's next design
                ready[qid] = (k + 1, pool.submit(densities, q, mask, f, k + 1))
        srv.step()
        for t in list(tickets):
            out = srv.poll(t)
            if out is None:
                continue
            qid, k = tickets.pop(t)
            busy.discard(qid)
            st, info, ms = out
            lat.append(ms)
            statuses.append(st)
            done_solves += 1
            p, q, mask, f = probs[qid]
            nx, ny, nz = q["nel"]
            ndof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
            dof_iters += ndof * sum(info["iters"][:q["nrhs"]])
            if st != 0:
                failed.append(dict(id=qid, solve=k, status=st, kind=q["kind"], nel=q["nel"],
                                   nsub=q["nsub"], nrhs=q["nrhs"], nlevels=q["nlevels"],
                                   iters=info["iters"][:q["nrhs"]],
                                   rel_res=info["rel_res"][:q["nrhs"]]))
                log(f"  request {qid} solve {k}: status {st} {failed[-1]}")
            if k + 1 >= args.session_solves:
                srv.release(p)
                p.close()
                del probs[qid]
        if not tickets and not ready and pending:
            time.sleep(max(0.0, min(0.01, pending[0]["arrival"] - (time.perf_counter() - t0))))
        elif not tickets:
            time.sleep(0.0005)  # only densities in preparation: leave the host threads the CPU
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    srv.close()
    pool.shutdown()
    lat_s = np.sort(lat)
    out = {
        "metric": "MGCG solves/s and DOF\u00b7CG-iter/s at 1e-8 rel. residual; p50/p99 solve latency",
        "value": round(done_solves / elapsed, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": done_solves, "warmup": 0, "ms_per_step": round(elapsed / done_solves * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": f"served mix: {n} requests (cantilever / MBB / torsion; meshes "
                               f"32x16x16 ... 128x64x64; n in 1,2,4; 1-4 load cases), Poisson "
                               f"arrivals at {rate:.2f} requests/s, {args.session_solves} "
                               f"warm-started solves per session, HBM budget {args.budget_gb} GB, "
                               f"{args.slots} slots",
                   "rtol": 1e-8},
        "p50_ms": round(float(np.percentile(lat_s, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_s, 99)), 3),
        "statuses": sorted(set(statuses)),
        "not_converged": len(failed),
        "dof_cg_iter_per_s": float(f"{dof_iters / elapsed:.4g}"),
        "elapsed_s": round(elapsed, 3),
        "rate": rate,
    }
    return out


PROJ_WORKLOAD = dict(nel=(64, 32, 32), nsub=4, ndes=2, rmin=1.5)


def proj_nnz(nel, n, d, rmin):
    """Nonzeros of W (pairs of density and design cells within rmin), counted
    per axis: the squared centre offsets m^2 (in units of 1/(2nd)^2) of every
    axis pair, then the triples with m_x^2 + m_y^2 + m_z^2 <= (2 n d rmin)^2."""
    R2 = (2.0 * n * d * rmin) ** 2

    def axis(ne):
        i = np.arange(ne * n)[:, None]
        j = np.arange(ne * d)[None, :]
        m2 = (((2 * i + 1) * d - (2 * j + 1) * n) ** 2).astype(np.float64)
        return m2[m2 <= R2]
    mz, my, mx = axis(nel[2]), axis(nel[1]), np.sort(axis(nel[0]))
    uz, cz = np.unique(mz, return_counts=True)
    uy, cy = np.unique(my, return_counts=True)
    total = 0
    for a, ca in zip(uz, cz):
        for b, cb in zip(uy, cy):
            if a + b <= R2:
                total += int(ca) * int(cb) * int(np.searchsorted(mx, R2 - a - b, side="right"))
    return total


def run_projection(args):
    import torch
    from paper_2311_05595_amd import api

    wl = PROJ_WORKLOAD
    nel, n, d, rmin = wl["nel"], wl["nsub"], wl["ndes"], wl["rmin"]
    dev = torch.device("cuda:0")
    pr = api.Projection(nel, n, d, rmin)
    gen = torch.Generator(device=dev).manual_seed(17)
    x = torch.rand(pr.nx, dtype=torch.float64, device=dev, generator=gen)
    g = torch.randn(pr.nrho, dtype=torch.float64, device=dev, generator=gen)
    rho = torch.empty(pr.nrho, dtype=torch.float64, device=dev)
    gx = torch.empty(pr.nx, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        pr.apply(x, out=rho)
        pr.apply_transpose(g, out=gx)
    torch.cuda.synchronize()

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_f = timed(lambda: pr.apply(x, out=rho), args.steps)
    t_t = timed(lambda: pr.apply_transpose(g, out=gx), args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pr.apply(x, out=rho)
        pr.apply_transpose(g, out=gx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nnz = proj_nnz(nel, n, d, rmin)
    flops = 2.0 * nnz                       # one multiply-add per nonzero of W
    bytes_f = 8.0 * (pr.nx + 2 * pr.nrho)   # x read, 1/omega read, rho written
    bytes_t = 8.0 * (2 * pr.nrho + pr.nx)   # g and 1/omega read, W^T g written

    def roof(t, nbytes):
        alu = flops / (PEAK_FP64_TFLOPS * 1e12) >= nbytes / (PEAK_HBM_GBS * 1e9)
        if alu:
            a, p, u = flops / t / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
        else:
            a, p, u = nbytes / t / 1e9, PEAK_HBM_GBS, "GB/s"
        return {"bound": "alu" if alu else "hbm", "achieved": round(a, 3), "peak": p, "unit": u,
                "frac": round(a / p, 4), "traffic": None, "avg_us": round(t * 1e6, 2),
                "alg_flop_per_launch": flops, "alg_bytes_per_launch": nbytes,
                "alg_GBs": round(nbytes / t / 1e9, 1)}
    out = {
        "metric": "design-variable projections/s (rho = W x and W^T g, one pair per step)",
        "value": round(args.steps / elapsed, 2), "unit": "projections/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"projection {nel[0]}x{nel[1]}x{nel[2]} elements, n={n} density "
                               f"and d={d} design cells per element, rmin={rmin}",
                   "n_rho": pr.nrho, "n_x": pr.nx, "nnz_W": nnz},
        "roofline": roof(t_f, bytes_f),
        "roofline_transpose": roof(t_t, bytes_t),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = proj_cpu_baseline(x.cpu().numpy(), pr, budget_s=args.cpu_budget)
    pr.close()
    print(json.dumps(out), flush=True)


def proj_cpu_baseline(x, pr, budget_s=10.0):
    """The oracle's plain single-entry projection timed on a bounded sample of
    density cells, scaled to one full projection (forward only)."""
    from oracle import projection as P
    wl = PROJ_WORKLOAD
    nel, n, d, rmin = wl["nel"], wl["nsub"], wl["ndes"], wl["rmin"]
    Sr = P.lattice_shape(nel, n)
    rng = np.random.default_rng(3)
    t0 = time.perf_counter()
    done = 0
    while time.perf_counter() - t0 < budget_s and done < 20000:
        flat = int(rng.integers(pr.nrho))
        P.project_at(x, (flat % Sr[2], (flat // Sr[2]) % Sr[1], flat // (Sr[2] * Sr[1])),
                     nel, n, d, rmin)
        done += 1
    dt = time.perf_counter() - t0
    per_proj = dt / done * pr.nrho
    return {"value": round(1.0 / per_proj, 8), "unit": "projections/s (forward)", "cores": 1,
            "kind": "oracle",
            "sample": f"oracle single-entry evaluation of rho_i for {done} random density cells "
                      f"in {dt:.1f} s on 1 host thread, scaled to all {pr.nrho} cells"}


def run_lp(args):
    import torch
    from paper_2311_05595_amd import api

    n = 64 * 32 * 32 * 8  # the design lattice of the 64x32x32 mesh, 2^3 cells per element
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 1.0, n)
    g = -rng.exponential(1.0, n)
    a = rng.uniform(0.5, 1.5, n) / 8.0
    delta = 0.05
    l, u = np.maximum(-delta, -x), np.minimum(delta, 1.0 - x)
    b = float(a @ l + 0.4 * (a @ (u - l)))
    dev = torch.device("cuda:0")
    gd, ad, xd = (torch.tensor(v, device=dev) for v in (g, a, x))
    sd = torch.empty(n, dtype=torch.float64, device=dev)
    lp = api.LP(n)
    for _ in range(args.warmup):
        lp.solve(gd, ad, xd, b, delta, out=sd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = lp.solve(gd, ad, xd, b, delta, out=sd)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    nbytes = 8.0 * 4 * n  # g, a, x read, s written
    out = {
        "metric": "SLP LP subproblem solves/s (volume constraint, trust region)",
        "value": round(1.0 / t, 1), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"LP step over {n} design variables (64x32x32 elements, 2^3 "
                               f"design cells each), delta={delta}", "feasible": info["feasible"]},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(nbytes / t / 1e9 / PEAK_HBM_GBS, 5),
                     "traffic": None, "avg_us": round(t * 1e6, 1), "alg_bytes_per_launch": nbytes,
                     "note": "whole call: 31 kernel launches (8 radix passes of 3) and one "
                             "host read of the result"},
    }
    if not args.no_cpu:
        from oracle import slp
        t1 = time.perf_counter()
        slp.lp_step(g, a, x, b, delta)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "solves/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the oracle's LP step on the same {n} variables, "
                                         f"once ({dt:.2f} s, 1 host thread)"}
    lp.close()
    print(json.dumps(out), flush=True)


def run_threshold(args):
    import torch
    from paper_2311_05595_amd import api

    n = 64 * 32 * 32 * 64  # the density lattice of the 64x32x32 mesh, 4^3 sub-elements each
    rng = np.random.default_rng(31)
    rho = np.clip(rng.beta(0.7, 1.2, n), 0.0, 1.0)
    vfrac, beta = 0.3, 8.0
    dev = torch.device("cuda:0")
    rd = torch.tensor(rho, device=dev)
    od = torch.empty(n, dtype=torch.float64, device=dev)
    lp = api.LP(n)

    def timed(fn):
        for _ in range(args.warmup):
            r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, r

    t_sel, _ = timed(lambda: lp.density_threshold(rd, vfrac, out=od))
    t_hv, (_, eta, iters) = timed(lambda: lp.heaviside(rd, beta, out=od))
    t_cos, _ = timed(lambda: lp.angle_cos(rd, od))
    gl = rng.standard_normal(n) * np.exp(2.0 * rng.standard_normal(n))
    rr = np.where(rho >= 0.95, 1.0, np.where(rho <= 0.05, 0.0, rho))
    rrd, gld = torch.tensor(rr, device=dev), torch.tensor(gl, device=dev)
    t_lg, (_, alpha_t) = timed(lambda: lp.lagrangian_threshold(rrd, gld, out=od))
    nbytes = 16.0 * n  # the densities read and the 0/1 design written
    out = {
        "metric": "density thresholdings/s (top-k rule of the density values)",
        "value": round(1.0 / t_sel, 1), "unit": "thresholdings/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_sel * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"thresholding of {n} densities (64x32x32 elements, 4^3 "
                               f"sub-elements each), v_frac={vfrac}",
                   "heaviside_ms": round(t_hv * 1e3, 4), "heaviside_beta": beta,
                   "heaviside_eta": eta, "heaviside_newton_iters": iters,
                   "angle_cos_ms": round(t_cos * 1e3, 4),
                   "lagrangian_ms": round(t_lg * 1e3, 4), "lagrangian_alpha": alpha_t},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / t_sel / 1e9, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(nbytes / t_sel / 1e9 / PEAK_HBM_GBS, 5), "traffic": None,
                     "avg_us": round(t_sel * 1e6, 1), "alg_bytes_per_launch": nbytes,
                     "note": "whole call: 29 kernel launches (8 radix passes of 3) and one "
                             "host read of the selection state"},
    }
    if not args.no_cpu:
        from oracle import threshold
        t1 = time.perf_counter()
        threshold.density_threshold(rho, vfrac)
        dt = time.perf_counter() - t1
        t2 = time.perf_counter()
        threshold.heaviside(rho, beta, threshold.eta_newton(rho, beta))
        dt2 = time.perf_counter() - t2
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "thresholdings/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's density-value rule on the same {n} "
                                         f"densities, once ({dt:.2f} s, 1 host thread); its "
                                         f"Heaviside projection with Newton's eta {dt2:.2f} s"}
    lp.close()
    print(json.dumps(out), flush=True)


def run_fixing(args):
    import torch
    import workloads as W
    from paper_2311_05595_amd import api

    nel, n, d, order = (64, 32, 32), 4, 2, 2
    rng = np.random.default_rng(41)
    # void, solid and mixed regions at the element scale
    from workloads import fields
    blobs = fields.gaussian_random_field((nel[2], nel[1], nel[0]), 41)
    lo, hi = np.quantile(blobs, [0.4, 0.7])
    up = lambda a, m: np.repeat(np.repeat(np.repeat(a, m, 0), m, 1), m, 2)
    kind = up(np.where(blobs < lo, 0, np.where(blobs > hi, 2, 1)), n)
    rho = np.where(kind == 0, 1e-7, np.where(kind == 2, 0.95, 0.5))
    grad = rng.uniform(-1e-6, 1e-6, (d * nel[2], d * nel[1], d * nel[0]))
    mask, _ = W.make_problem("cantilever", *nel, order, 1)
    dev = torch.device("cuda:0")
    rd, gd = torch.tensor(rho, device=dev), torch.tensor(grad, device=dev)
    m0 = torch.tensor(mask, device=dev)
    dm = m0.clone()
    for _ in range(args.warmup):
        dm.copy_(m0)
        api.fix_variables(nel, n, d, order, rd, gd, dm)
    torch.cuda.synchronize()
    t = 0.0
    for _ in range(args.steps):
        dm.copy_(m0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, cnt = api.fix_variables(nel, n, d, order, rd, gd, dm)
        t += time.perf_counter() - t0
    t /= args.steps
    nn = (order * nel[0] + 1) * (order * nel[1] + 1) * (order * nel[2] + 1)
    nelt = nel[0] * nel[1] * nel[2]
    nbytes = 8.0 * rho.size + 8.0 * grad.size + nelt + grad.size + 3.0 * nn
    out = {
        "metric": "fixings/s (void and solid elements, fixed design variables, suppressed Q2 DOFs)",
        "value": round(1.0 / t, 1), "unit": "fixings/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"64x32x32 elements, 4^3 densities and 2^3 design cells each, "
                               f"Q2 lattice {2 * nel[0] + 1}x{2 * nel[1] + 1}x{2 * nel[2] + 1}",
                   "counts": cnt},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / t / 1e9, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(nbytes / t / 1e9 / PEAK_HBM_GBS, 5),
                     "traffic": None, "avg_us": round(t * 1e6, 1), "alg_bytes_per_launch": nbytes,
                     "note": "whole call: 8 launches, one scratch allocation and one read-back"},
    }
    if not args.no_cpu:
        from oracle import fixing
        t1 = time.perf_counter()
        fk = fixing.surrounded(fixing.classify(rho, grad, nel, n, d))
        fixing.dof_mask(mask, fixing.suppressed_nodes(fk, order))
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "fixings/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the oracle on the same lattices, once ({dt:.2f} s, "
                                         f"1 host thread)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--smoother", default=None, choices=[None, "jacobi", "gauss-seidel"],
                    help="finest-level smoother (default: the workload's)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--launch", default="eager", choices=["eager", "graph", "fused"],
                    help="how the solve is launched (fused: one launch per solve, small "
                         "trilinear FP64 workloads only; no per-kernel roofline then)")
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=60.0,
                    help="seconds of oracle CG iterations for the reference solve")
    ap.add_argument("--no-served", action="store_true",
                    help="default line without the served FP64-vs-mixed legs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--projection", action="store_true",
                    help="time the design-variable projection and its transpose")
    ap.add_argument("--lp", action="store_true", help="time the SLP step's LP subproblem")
    ap.add_argument("--fixing", action="store_true",
                    help="time the choice of fixed variables before the degree is raised")
    ap.add_argument("--threshold", action="store_true",
                    help="time the density thresholding and the Heaviside projection")
    ap.add_argument("--batch", type=int, default=0, metavar="N",
                    help="time N small (c1) problems solved eagerly one by one and in one "
                         "fused multi-problem launch")
    ap.add_argument("--batch-modes", default="eager,fused",
                    help="--batch: the launch modes to time, comma-separated")
    ap.add_argument("--apply-sweep", action="store_true",
                    help="time the matrix-free CG apply on lattices of 0.7M to 8.6M DOF")
    ap.add_argument("--requests", type=int, default=256, help="c5: number of requests")
    ap.add_argument("--session-solves", type=int, default=5, help="c5: solves per session")
    ap.add_argument("--rate", type=float, default=0.0, help="c5: arrivals per second")
    ap.add_argument("--budget-gb", type=float, default=48.0, help="c5: HBM budget")
    ap.add_argument("--slots", type=int, default=16, help="c5: concurrent solves")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.apply_sweep:
        apply_sweep(args)
        return
    if args.batch:
        batch_bench(args)
        return
    if args.fixing:
        if args.gpus != 1:
            print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
            sys.exit(2)
        run_fixing(args)
        return
    if args.threshold:
        if args.gpus != 1:
            print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
            sys.exit(2)
        run_threshold(args)
        return
    if args.lp:
        if args.gpus != 1:
            print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
            sys.exit(2)
        run_lp(args)
        return
    if args.projection:
        if args.gpus != 1:
            print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
            sys.exit(2)
        run_projection(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (a multi-GPU run is not supported); --gpus must be 1"}))
        sys.exit(2)
    if args.config == "c5":
        run_served(args)
        return
    run(args)


if __name__ == "__main__":
    main()
