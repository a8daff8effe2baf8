"""Benchmark: time to a relative residual of 1e-8 on the 1024 x 1024 Shishkin
mesh at eps = 1e-6, FP64 and mixed precision, on one MI355X.

A step is one FP64 solve followed by one mixed-precision solve of the same
problem (boundary-layer-preconditioned FGMRES(50), zero initial guess, inputs
resident on the device).  Setup (preconditioner construction) is timed once,
apart.  The JSON line carries the per-kernel roofline of the dominant kernel
(HIP events recorded by the library on its stream over the timed steps) and
the CPU oracle timed on this host.

The default run also measures, in the same JSON line:
  batch       64 uneven instances solved together (mixed, 1e-8): solves/s;
  multi_rhs   N = 2048, eps = 1e-6, 16 right-hand sides: mixed solves and the
              adjoint solves of their gradients;
  oned        the 1D method for 2048 problems in one launch: solves/s;
  parabolic   one parabolic and one exponential layer, the paper's test at
              N = 2048, eps = 1e-7: ms per solve;
  copy        the attainable HBM bandwidth of a plain 1 GiB device copy;
each with its own roofline entry and CPU-oracle baseline.  --workload runs
one of them alone (its own JSON line).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--eps E] [--no-cpu]
                       [--workload all|headline|batch|multi_rhs|oned|parabolic|copy_probe]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time to rel-res 1e-8, 1024^2 eps=1e-6 (FP64 vs mixed) + HBM GB/s %peak"
HBM_PEAK_GBS = 8000.0
# kernels behind each timing class in the mixed solve at this size
KERNEL_NAMES = {"sweep": "k_sweep<float, false, 16, *, *> (all sweeps: interior and corner "
                         "levels 512/256/128)",
                "gs_rhs": "k_gs_rhs / k_mg_prolong_gs<float, false>",
                "lines": "k_lines<float, false, 8, 1, 4>", "spmv": "k_stencil<float, ...>"}
# measured HBM traffic of the sweep launches (two rocprofv3 --pmc runs,
# FETCH_SIZE then WRITE_SIZE, scaled by a plain copy of known size), valid
# while the sweep source is the one it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_traffic.txt")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2108_13468_amd", "csrc", "kernels_sweep.h")
# worker pool of the CPU baselines: the host's cores available to this
# process, at most 16 (one GPU's share of a shared host)
POOL_MAX = 16


def measured_traffic():
    """Bytes per sweep launch from the committed counter summary, or None when
    it is missing or was taken on a different kernel source."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
        if kv.get("kernel_source_sha256") != sha:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def host_info():
    """Cores this process may use (the pool size of the CPU baselines) and
    the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": avail, "pool": min(POOL_MAX, avail), "cpu_model": model}


def copy_probe(args):
    """A plain device copy of known size (counter calibration for the
    traffic figure): 256 MiB read, 256 MiB written, three times."""
    import torch
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_probe_bytes_read": x.numel() * 4, "copy_probe_bytes_written": y.numel() * 4}


def copy_bandwidth():
    """Attainable HBM bandwidth: a 1 GiB device-to-device copy (read plus
    write bytes over the event time, median of 10)."""
    import numpy as np
    import torch
    n = 1 << 28  # 1 GiB of float32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    ts = []
    for _ in range(10):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    gbs = 2.0 * n * 4 / (ms * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_copied": n * 4, "ms": round(ms, 3), "GBps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}


def roofline_of(kt, names=None, prefer=None, traffic=None):
    """Roofline entry of the dominant kernel class (or `prefer`) of a timing
    dictionary {class: (ms, launches, algorithmic bytes)}: algorithmic bytes
    per launch over the average launch duration."""
    dom = prefer or max(kt, key=lambda k: kt[k][0])
    ms, nl, by = kt[dom]
    avg_us = 1e3 * ms / max(nl, 1)
    bpl = by / max(nl, 1)
    achieved = bpl / (avg_us * 1e-6) / 1e9 if nl else 0.0
    out = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
           "kernel": (names or {}).get(dom, dom), "avg_launch_us": round(avg_us, 3),
           "launches": nl, "bytes_per_launch": round(bpl, 1)}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / bpl, 3)
    return out


def kernels_of(kt, steps):
    return {k: {"ms": round(v[0] / steps, 3), "launches": v[1] // steps,
                "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else 0.0,
                "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 2) if v[0] > 0 else 0.0}
            for k, v in kt.items()}


def pool_map(fn, items, cores):
    """fn over items with `cores` threads (the oracle's C calls release the
    interpreter lock); returns (results, wall seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=max(1, min(cores, len(items)))) as ex:
        res = list(ex.map(fn, items))
    return res, time.perf_counter() - t0


def unscaled_rel_res(gp, F, U):
    """||F - A U||_2 / ||F||_2 with the library's FP64 operator."""
    import torch
    r = F - gp.apply("A", U)
    return float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(F))


def headline(args):
    import numpy as np
    import torch
    from paper_2108_13468_amd import blp, inputs

    inst = inputs.plain(args.N, args.eps, seed=1)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    gp = blp.from_instance(inst)
    e0, e1 = ev(), ev()
    e0.record(stream)
    gp.precondition()
    e1.record(stream)
    torch.cuda.synchronize()
    setup_ms = e0.elapsed_time(e1)
    F = gp.sine_rhs(inst.a)
    opts = dict(tol=1e-8, scaled=True, restart=50, maxit=2000)

    for _ in range(args.warmup):
        gp.solve(F, precision="fp64", **opts)
        gp.solve(F, precision="mixed", **opts)
    torch.cuda.synchronize()

    # Timed steps: one event pair around each solve, nothing between kernels.
    t_fp64, t_mixed = [], []
    ts, te = ev(), ev()
    ts.record(stream)
    for _ in range(args.steps):
        a, b, c = ev(), ev(), ev()
        a.record(stream)
        U64, i64 = gp.solve(F, precision="fp64", **opts)
        b.record(stream)
        U32, i32 = gp.solve(F, precision="mixed", **opts)
        c.record(stream)
        torch.cuda.synchronize()
        t_fp64.append(a.elapsed_time(b))
        t_mixed.append(b.elapsed_time(c))
        i64, i32 = i64[0], i32[0]
    te.record(stream)
    torch.cuda.synchronize()
    total_ms = ts.elapsed_time(te)

    # The same steps again with the library's per-kernel events (an event pair
    # around every launch, on the launch's stream): kernel durations for the
    # roofline.  The events add gaps between kernels, so this pass does not
    # give the solve time.  Each precision has its own accumulation window,
    # so a class average is the average of one kernel template.
    acc = {"fp64": {}, "mixed": {}}
    ev_ms = {"fp64": [], "mixed": []}
    for _ in range(args.steps):
        for prec in ("fp64", "mixed"):
            gp.timing(True)
            a, b = ev(), ev()
            a.record(stream)
            gp.solve(F, precision=prec, **opts)
            b.record(stream)
            for k, v in gp.timing(False).items():
                q = acc[prec].setdefault(k, [0.0, 0, 0.0])
                for r in range(3):
                    q[r] += v[r]
            ev_ms[prec].append(a.elapsed_time(b))

    fp64_ms = float(np.median(t_fp64))
    mixed_ms = float(np.median(t_mixed))
    # dominant kernel of the mixed solve (the headline value)
    km = {k: tuple(v) for k, v in acc["mixed"].items()}
    dom = max(km, key=lambda k: km[k][0])
    roofline = roofline_of(km, KERNEL_NAMES, traffic=measured_traffic() if dom == "sweep" else None)
    roofline["kernel"] += " (mixed solve)"
    avg_us = roofline["avg_launch_us"]
    nl = km[dom][1]
    # Second bound of the single-right-hand-side sweeps: their dependency
    # chain.  A sweep of an n x n rectangle is 2n - 1 anti-diagonals, each a
    # dependent step.  Per preconditioner apply of the mixed solve: the
    # interior (m = N - 1 - N/2) once, and the corner levels above the
    # LDS-resident cycle (N/2, N/4, .. while above 64 nodes and even) twice
    # per corner cycle.
    latency = None
    if dom == "sweep":
        applies = i32["iterations"]
        cycles = 0.5 * (i32["mg_cycles_min"] + i32["mg_cycles_max"])
        m = args.N - 1 - args.N // 2
        lv, n = [], args.N // 2
        while n > 64 and n % 2 == 0:
            lv.append(n)
            n //= 2
        per_apply = [(2 * m - 1, 1.0)] + [(2 * q - 1, 2.0 * cycles) for q in lv]
        launches = applies * sum(c for _, c in per_apply)
        steps = applies * sum(st * c for st, c in per_apply)
        per_launch = steps / launches
        latency = {"kernel": roofline["kernel"],
                   "chain": "2n - 1 dependent anti-diagonal steps per n x n sweep",
                   "launches_modelled": round(launches, 1),
                   "launches_measured": round(nl / args.steps, 1),  # per solve
                   "dependent_steps_per_launch": round(per_launch, 1),
                   "ns_per_step": round(1e3 * avg_us / per_launch, 2),
                   "cycles_per_step_at_2.4GHz": round(2.4 * 1e3 * avg_us / per_launch, 1)}
    kernels = {prec: kernels_of({k: tuple(v) for k, v in acc[prec].items()}, args.steps)
               for prec in acc}

    out = {
        "metric": METRIC,
        "value": round(mixed_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "N=%d per side (%d unknowns), eps=%g, c=(1+x^2, 1+y), r=1, "
                               "seeded 3x3 sine-series f, FGMRES(50) to relative residual 1e-8 "
                               "of the Jacobi-scaled system" % (args.N, (args.N - 1) ** 2, args.eps),
                   "N": args.N, "eps": args.eps},
        "fp64_ms": round(fp64_ms, 3),
        "mixed_ms": round(mixed_ms, 3),
        "ms_with_kernel_events": {k: round(float(np.median(v)), 3) for k, v in ev_ms.items()},
        "setup_ms": round(setup_ms, 3),
        "iterations": {"fp64": i64["iterations"], "mixed": i32["iterations"],
                       "mixed_restarts": i32["restarts"],
                       "corner_cycles": [i64["mg_cycles_min"], i64["mg_cycles_max"]]},
        # the stopping test is on the Jacobi-scaled system; the plain
        # residual of the same iterates is reported beside it
        "rel_res": {"fp64": i64["res"] / i64["norm_F"], "mixed": i32["res"] / i32["norm_F"]},
        "rel_res_unscaled": {"fp64": unscaled_rel_res(gp, F, U64),
                             "mixed": unscaled_rel_res(gp, F, U32)},
        "footprint_bytes": gp.footprint(),
        "roofline": roofline,
        "latency": latency,
        "kernels_per_step": kernels,
        "paper_context": {"seconds": 0.921, "iterations": 5,
                          "hardware": "one core of a 2.4 GHz Xeon, serial C",
                          "stopping": "||R||_2 <= 10 ln(N)/N (absolute), sigma = 5/2, "
                                      "manufactured solution (Table 7)"},
    }

    if not args.no_cpu:
        from oracle import oracle as O
        op = O.Problem(inst.N, inst.eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const)
        Fo = O.sine_series(inst.N, op.x, op.y, inst.a)
        t0 = time.perf_counter()
        uo, st, info_o, _ = op.fgmres(Fo, tol=1e-8, scaled=True, maxit=2000)
        cpu_ms = 1e3 * (time.perf_counter() - t0)
        ut, _, _, _ = op.fgmres(Fo, tol=1e-10, scaled=True, maxit=2000)
        scale = np.abs(ut).max()
        hi = host_info()
        out["cpu_baseline"] = {"value": round(cpu_ms, 1), "unit": "ms", "cores": 1,
                               "kind": "oracle",
                               "sample": "one FP64 solve of the same problem to the same "
                                         "tolerance (plain C oracle, single thread, %d "
                                         "iterations)" % info_o.iterations,
                               "cpu_model": hi["cpu_model"], "nproc": hi["nproc"]}
        out["err_vs_oracle"] = {
            "fp64": float(np.abs(U64.cpu().numpy() - ut).max() / scale),
            "mixed": float(np.abs(U32.cpu().numpy() - ut).max() / scale),
            "reference": "oracle FGMRES to scaled relative residual 1e-10, max-norm relative"}
    return out


def batch(args):
    """64 uneven instances solved together (mixed precision, 1e-8): solves/s."""
    import numpy as np
    import torch
    from paper_2108_13468_amd import blp, inputs
    insts = inputs.batch_cases(64)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ps = [blp.from_instance(i).precondition() for i in insts]
    F = [p.sine_rhs(i.a) for p, i in zip(ps, insts)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = blp.Batch(ps, graphs=True, autotune=True)
    opts = dict(tol=1e-8, precision="mixed", maxit=2000)
    steps, warmup = args.side_steps, args.side_warmup
    for _ in range(warmup):
        b.solve(F, **opts)
    a, c = ev(), ev()
    a.record()
    for _ in range(steps):
        U, info = b.solve(F, **opts)
    c.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(c) / steps
    b.timing(True)
    b.solve(F, **opts)
    kt = b.timing(False)
    it = [d["iterations"] for d in info]
    out = {"metric": "batched solves/s, 64 uneven instances (N in {128..1024}, eps in [1e-8,1e-2]), "
                     "mixed, rel-res 1e-8",
           "value": round(64e3 / ms, 3), "unit": "solves/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "64 instances drawn by the uneven-batch recipe (seed 2): N "
                                  "uniform in {128,256,512,1024}, log10 eps uniform in [-8,-2], "
                                  "c=(1+ax,1+by), r uniform in [0.5,2], 3x3 sine f; one batch "
                                  "(graphs, autotuned), FGMRES(50) mixed to 1e-8",
                      "classes": {str(N): sum(1 for i in insts if i.N == N)
                                  for N in (128, 256, 512, 1024)}},
           "converged": sum(d["converged"] for d in info),
           "iterations": {"min": min(it), "max": max(it), "mean": round(float(np.mean(it)), 2)},
           # the instances with the most iterations set the batch's sequential chain
           "hardest": [{"N": insts[k].N, "eps": float("%.3g" % insts[k].eps), "iterations": it[k],
                        "corner_cycles": [info[k]["mg_cycles_min"], info[k]["mg_cycles_max"]]}
                       for k in sorted(range(len(it)), key=lambda k: -it[k])[:3]],
           "setup_s": round(setup_s, 3), "footprint_bytes": b.footprint(),
           "roofline": roofline_of(kt), "kernels_per_solve": kernels_of(kt, 1),
           "tuning": b.describe()}
    if not args.no_cpu:
        from oracle import oracle as O
        hi = host_info()

        def solve(k):
            i = insts[k]
            t = time.perf_counter()
            op = O.Problem(i.N, i.eps, c1=i.c1_at, c2=i.c2_at, r=i.r_const)
            _, st, io, _ = op.fgmres(O.sine_series(i.N, op.x, op.y, i.a), tol=1e-8, scaled=True,
                                     maxit=2000)
            return time.perf_counter() - t, io.iterations

        # every N <= 256 instance is solved (measured); N = 512 and 1024 are
        # extrapolated from the first two instances of each class: their
        # seconds per iteration times each instance's iteration count (the
        # GPU run's, the same algorithm)
        small = [k for k, i in enumerate(insts) if i.N <= 256]
        sample = {N: [k for k, i in enumerate(insts) if i.N == N][:2] for N in (512, 1024)}
        res, wall_small = pool_map(solve, small + sample[512] + sample[1024], hi["pool"])
        t_of = dict(zip(small + sample[512] + sample[1024], res))
        per_it = {N: sum(t_of[k][0] for k in ks) / max(1, sum(t_of[k][1] for k in ks))
                  for N, ks in sample.items()}
        est = [t_of[k][0] if k in small else it[k] * per_it[insts[k].N] for k in range(64)]
        cpu_s = sum(est)
        wall = max(max(est), cpu_s / hi["pool"])
        out["cpu_baseline"] = {
            "value": round(64 / wall, 3), "unit": "solves/s", "cores": hi["pool"],
            "kind": "oracle",
            "sample": "all 40 instances with N <= 256 solved by the FP64 oracle (one solve per "
                      "core, %.1f s wall); the 24 with N = 512 and 1024 extrapolated from the "
                      "first two of each class (%.3f and %.3f s per iteration) times their "
                      "iteration counts; value = 64 / max(longest solve, total CPU seconds / "
                      "cores) = 64 / %.1f s" % (wall_small, per_it[512], per_it[1024], wall),
            "cpu_seconds_total": round(cpu_s, 1), "cpu_model": hi["cpu_model"],
            "nproc": hi["nproc"]}
    return out


def multi_rhs(args):
    """N = 2048, eps = 1e-6, 16 right-hand sides: mixed forward solves plus the
    16 adjoint solves of the misfits' gradients."""
    import numpy as np
    import torch
    from paper_2108_13468_amd import blp, inputs
    inst, A = inputs.multi_rhs_case()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    p = blp.from_instance(inst).precondition()
    F = [p.sine_rhs(A[k]) for k in range(A.shape[0])]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = blp.Batch([p] * len(F), graphs=True, autotune=True)
    opts = dict(tol=1e-8, precision="mixed", maxit=2000)

    def step():
        U, i1 = b.solve(F, **opts)
        G = [u.clone() for u in U]  # dJ/du of J = 0.5 ||u||^2 per right-hand side
        L, i2 = b.solve_adjoint(G, **opts)
        # dJ/da, the gradient with respect to each misfit's 3 x 3 sine
        # coefficients (allocation-free projections of the adjoint solutions)
        g = [p.sine_project_noalloc(lam, A.shape[2], A.shape[1]) for lam in L]
        return i1, i2, g
    steps, warmup = args.side_steps, args.side_warmup
    for _ in range(warmup):
        step()
    a, c = ev(), ev()
    a.record()
    for _ in range(steps):
        i1, i2, grads = step()
    c.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(c) / steps
    b.timing(True)
    step()
    kt = b.timing(False)
    by_kernel = {k: roofline_of(kt, prefer=k) for k in ("spmv", "sweep", "lines", "mg_other",
                                                          "krylov")}
    out = {"metric": "16 right-hand sides at N=2048, eps=1e-6: mixed solves + adjoint gradients "
                     "(dJ/d sine coefficients of all 16 misfits)",
           "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "N=2048 (4.19M unknowns), eps=1e-6, c=(1+x^2,1+y), r=1, 16 "
                                  "seeded 3x3 sine right-hand sides; 16 FGMRES(50) mixed solves "
                                  "to 1e-8, 16 adjoint solves and the 16 projections dJ/da "
                                  "(J = 0.5 ||u||^2 per right-hand side), one batch (graphs, "
                                  "autotuned)"},
           "gradient_norms": [round(float((g ** 2).sum() ** 0.5), 6) for g in grads],
           "iterations": {"forward": [d["iterations"] for d in i1],
                          "adjoint": [d["iterations"] for d in i2]},
           "corner_cycles": {"forward": [min(d["mg_cycles_min"] for d in i1),
                                         max(d["mg_cycles_max"] for d in i1)],
                             "adjoint": [min(d["mg_cycles_min"] for d in i2),
                                         max(d["mg_cycles_max"] for d in i2)]},
           "setup_s": round(setup_s, 3),
           "footprint_bytes": {"batch": b.footprint(), "problem": p.footprint()},
           "roofline": roofline_of(kt),
           "roofline_by_kernel": by_kernel,
           "kernels_per_step": kernels_of(kt, 1), "tuning": b.describe()}
    if not args.no_cpu:
        from oracle import oracle as O
        hi = host_info()
        op = O.Problem(inst.N, inst.eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const)
        Fo = [O.sine_series(inst.N, op.x, op.y, A[k]) for k in range(A.shape[0])]

        def fwd(k):
            t = time.perf_counter()
            _, _, io, _ = op.fgmres(Fo[k], tol=1e-8, scaled=True, maxit=2000)
            return time.perf_counter() - t, io.iterations

        # the 16 forward solves, one per core (measured); the adjoint solves
        # extrapolated from two iterations of the first one
        res, wall_f = pool_map(fwd, list(range(len(Fo))), hi["pool"])
        t = time.perf_counter()
        _, _, ia, _ = op.fgmres(Fo[0], tol=1e-8, scaled=True, maxit=2, transpose=True)
        per_it_adj = (time.perf_counter() - t) / max(1, ia.iterations)
        adj = [d["iterations"] * per_it_adj for d in i2]
        wall_a = max(max(adj), sum(adj) / hi["pool"])
        out["cpu_baseline"] = {
            "value": round(1e3 * (wall_f + wall_a), 1), "unit": "ms", "cores": hi["pool"],
            "kind": "oracle",
            "sample": "the 16 forward FP64 oracle solves, one per core (measured, %.1f s wall); "
                      "the 16 adjoint solves extrapolated from two iterations of the first "
                      "(%.2f s per iteration) times the adjoint iteration counts, spread over "
                      "the cores (%.1f s)" % (wall_f, per_it_adj, wall_a),
            "cpu_model": hi["cpu_model"], "nproc": hi["nproc"]}
    return out


def oned(args):
    """The 1D method (Sec. 2) for 2048 independent problems in one launch:
    the paper's test problem (c = 2 + sin 5x, r = 1, f = 4 exp(-x)) with N
    uniform in {128, ..., 2048} and log10 eps uniform in [-8, -4], M on the
    left, ||F - A u||_inf <= ||U^E||_inf ln(N)/N: solves/s."""
    import numpy as np
    import torch
    from paper_2108_13468_amd import blp
    rng = np.random.default_rng(5)
    S = 2048
    Ns = rng.choice([128, 256, 512, 1024, 2048], size=S)
    epss = 10.0 ** rng.uniform(-8.0, -4.0, size=S)
    probs, F = [], []
    for N, eps in zip(Ns, epss):
        _, x, _ = blp.mesh(int(N), float(eps), 2.0, (0.99, 0.99))
        probs.append(dict(N=int(N), eps=float(eps), c=2.0 + np.sin(5.0 * x), r=np.ones(N + 1),
                          clow=0.99))
        F.append(torch.as_tensor(4.0 * np.exp(-x[1:-1]), device="cuda"))
    steps, warmup = args.side_steps, args.side_warmup
    for _ in range(warmup):
        blp.solve_1d(probs, F, maxit=100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        U, info = blp.solve_1d(probs, F, maxit=100)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    it = np.array([d["iterations"] for d in info])
    # algorithmic bytes of the basis traffic: per iteration j (0-based) the
    # modified Gram-Schmidt reads j + 1 basis vectors twice and the update
    # reads j + 1 more; the operator, M^{-1} and residual stream about 12
    # vectors; 8 bytes per value, n = N - 1
    nbytes = sum(8.0 * (N - 1) * sum(3 * (j + 1) + 12 for j in range(k)) for N, k in zip(Ns, it))
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"metric": "1D method: batched solves/s, 2048 problems in one launch",
           "value": round(S * 1e3 / ms, 1), "unit": "solves/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2048 instances of -eps u'' - (2 + sin 5x) u' + u = 4 exp(-x) on "
                                  "Shishkin meshes (Clow = 0.99): N uniform in {128..2048}, log10 "
                                  "eps uniform in [-8, -4]; unrestarted GMRES with M of eq. block_M "
                                  "on the left, one workgroup per problem, one launch per batch "
                                  "(host set-up and copies included)"},
           "converged": int(sum(d["converged"] for d in info)),
           "iterations": {"min": int(it.min()), "max": int(it.max()), "mean": round(float(it.mean()), 2)},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                        "kernel": "k_gmres1d (whole call)",
                        "note": "one workgroup per problem: latency of block reductions and scans, "
                                "not bandwidth, sets the pace"}}
    if not args.no_cpu:
        from oracle import oracle as O
        hi = host_info()

        def solve(k):
            N, eps = int(Ns[k]), float(epss[k])
            p = O.Problem1D(N, eps, lambda x: 2.0 + np.sin(5.0 * x), 1.0, clow=0.99)
            Fo = 4.0 * np.exp(-p.x[1:-1])
            K = np.abs(p.solve(Fo)).max()
            p.gmres(Fo, K=K, g=np.log(N) / N, maxit=100)

        _, wall = pool_map(solve, list(range(S)), hi["pool"])
        out["cpu_baseline"] = {"value": round(S / wall, 1), "unit": "solves/s", "cores": hi["pool"],
                               "kind": "oracle",
                               "sample": "all 2048 problems, one FP64 oracle solve per core "
                                         "(direct solve for K, then GMRES), %.2f s wall" % wall,
                               "cpu_model": hi["cpu_model"], "nproc": hi["nproc"]}
    return out


def parabolic(args):
    """One parabolic and one exponential layer (Sec. 3.3): the paper's test
    problem -eps Lap u - u_x + u = f (eq. parabolic_MMS) on its largest mesh,
    N = 2048, eps = 1e-7, sigma = 5/2, Clow = 0.99; a step is one FP64 solve
    to the paper's stopping rule (||R||_2 <= 10 ln N / N, estimate test), and
    the same problem is also solved to rel-res 1e-8 (scaled system) in FP64
    and mixed precision.  The paper reports 3.525 s (5 iterations) for this
    solve on one 2.4 GHz Xeon core (Table 4): context, other hardware."""
    import numpy as np
    import torch
    from paper_2108_13468_amd import blp, inputs
    from tests.mms import parabolic_mms
    N, eps = 2048, 1e-7
    inst = inputs.mms_parabolic(N, eps)
    gp = blp.from_instance(inst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gp.precondition()
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    x, y = gp.nodes()
    u, f = parabolic_mms(eps, x, y)
    F = torch.as_tensor(f, device="cuda")
    tol = 10 * np.log(N) / N
    steps, warmup = args.side_steps, args.side_warmup

    def paper_solve():
        return gp.solve(F, tol=tol, absolute=True, scaled=False, stop_on_estimate=True)

    for _ in range(warmup):
        paper_solve()
    torch.cuda.synchronize()
    gp.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        U, info = paper_solve()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    kt = gp.timing(False)
    err = float(np.abs(U.cpu().numpy() - u).max())
    rel = {}
    for prec in ("fp64", "mixed"):
        gp.solve(F, tol=1e-8, scaled=True, precision=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Ur, ir = gp.solve(F, tol=1e-8, scaled=True, precision=prec)
        torch.cuda.synchronize()
        rel[prec] = {"ms": round(1e3 * (time.perf_counter() - t1), 3),
                     "iterations": ir[0]["iterations"],
                     "corner_cycles": [ir[0]["mg_cycles_min"], ir[0]["mg_cycles_max"]],
                     "rel_res_unscaled": unscaled_rel_res(gp, F, Ur)}
    roof = roofline_of(kt, names={"sweep": "k_par_wave<double, *, *, *> and k_sweep<double, ...> "
                                           "(the corner levels' Gauss-Seidel sweeps)"},
                       prefer="sweep")
    roof["note"] = ("wavefront Gauss-Seidel on levels of 1024 rows, one workgroup per system "
                    "and level: h + nx/M - 1 dependent steps per sweep, each step's instruction "
                    "issue in one wave, not bandwidth, sets the pace")
    out = {"metric": "parabolic case: solve time, N=2048, eps=1e-7, the paper's stopping rule",
           "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "-eps Lap u - u_x + u = f with the manufactured solution of eq. "
                                  "parabolic_MMS, N=2048 per side (4.19M unknowns), eps=1e-7, "
                                  "sigma=5/2, Clow=0.99 (tau_x = sigma eps ln N / Clow, tau_y = "
                                  "sigma sqrt(eps) ln N); FGMRES(50) until ||R||_2 <= 10 ln N / N "
                                  "(estimate test); corner: x-semicoarsening Galerkin multigrid "
                                  "to a 1e2 reduction"},
           "iterations": info[0]["iterations"],
           "corner_cycles": [info[0]["mg_cycles_min"], info[0]["mg_cycles_max"]],
           "max_error_vs_exact": err, "table3_error": 3.783e-3, "table4_iterations": 5,
           "setup_ms": round(setup_ms, 3),
           "rel_res_1e-8": rel,
           "paper_context": {"seconds": 3.525, "iterations": 5,
                             "hardware": "one core of a 2.4 GHz Xeon (Sec. 3.3, Table 4)"},
           "kernels": kernels_of(kt, steps), "roofline": roof}
    if not args.no_cpu:
        from oracle import oracle as O
        hi = host_info()
        p = O.Problem(N, eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const, sigma=inst.sigma,
                      clow_x=inst.clow[0], clow_y=inst.clow[1], y_layer="parabolic")
        uo, fo = parabolic_mms(eps, p.x, p.y)
        t0 = time.perf_counter()
        _, _, io, _ = p.fgmres(fo, tol=tol, absolute=True, mg_rtol=1e-2, stop_on_estimate=True)
        wall = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(1e3 * wall, 1), "unit": "ms", "cores": 1,
                               "kind": "oracle",
                               "sample": "the same solve by the FP64 oracle, one core "
                                         "(%d iterations)" % io.iterations,
                               "cpu_model": hi["cpu_model"], "nproc": hi["nproc"]}
    gp.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side-steps", type=int, default=3,
                    help="timed solves of the batch and multi-RHS workloads")
    ap.add_argument("--side-warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=("all", "headline", "batch", "multi_rhs", "oned",
                                           "parabolic", "copy_probe"), default="all")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (instances and "
              "right-hand sides shard without communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "all":
        out = headline(args)
        print("headline done", file=sys.stderr, flush=True)
        out["batch"] = batch(args)
        print("batch done", file=sys.stderr, flush=True)
        out["multi_rhs"] = multi_rhs(args)
        print("multi_rhs done", file=sys.stderr, flush=True)
        out["oned"] = oned(args)
        print("oned done", file=sys.stderr, flush=True)
        out["parabolic"] = parabolic(args)
        print("parabolic done", file=sys.stderr, flush=True)
        out["copy_bandwidth"] = copy_bandwidth()
    else:
        out = {"headline": headline, "batch": batch, "multi_rhs": multi_rhs, "oned": oned,
               "parabolic": parabolic, "copy_probe": copy_probe}[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
