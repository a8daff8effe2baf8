"""Benchmark: time to a relative residual of 1e-8 on the 1024 x 1024 Shishkin
mesh at eps = 1e-6, FP64 and mixed precision, on one MI355X.

A step is one FP64 solve followed by one mixed-precision solve of the same
problem (boundary-layer-preconditioned FGMRES(50), zero initial guess, inputs
resident on the device).  Setup (preconditioner construction) is timed once,
apart.  The JSON line carries the per-kernel roofline of the dominant kernel
(HIP events recorded by the library on its stream over the timed steps) and
the CPU oracle timed on this host.

Two further workloads print their own line when asked for (--workload):
  batch      64 uneven instances solved together (mixed, 1e-8): solves/s;
  multi_rhs  N = 2048, eps = 1e-6, 16 right-hand sides: mixed solves and the
             adjoint solves of their gradients.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--eps E] [--no-cpu]
                       [--workload headline|batch|multi_rhs]
"""
import argparse
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
SWEEP_SOURCE = os.path.join(ROOT, "paper_2108_13468_amd", "csrc", "kernels_prec.h")


def measured_traffic():
    """Bytes per sweep launch from the committed counter summary, or None when
    it is missing or was taken on a different kernel source."""
    import hashlib
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


def copy_probe(args):
    """A plain device copy of known size (counter calibration for the
    traffic figure): 256 MiB read, 256 MiB written, three times."""
    import torch
    x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": x.numel() * 4, "copy_probe_bytes_written": y.numel() * 4}))


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

    def step():
        U64, i64 = gp.solve(F, precision="fp64", **opts)
        U32, i32 = gp.solve(F, precision="mixed", **opts)
        return U64, i64[0], U32, i32[0]

    for _ in range(args.warmup):
        step()
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
    km = acc["mixed"]
    dom = max(km, key=lambda k: km[k][0])
    ms, nl, by = km[dom]
    avg_us = 1e3 * ms / max(nl, 1)
    achieved = (by / max(nl, 1)) / (avg_us * 1e-6) / 1e9 if nl else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": measured_traffic() if dom == "sweep" else None,
                "kernel": KERNEL_NAMES.get(dom, dom) + " (mixed solve)",
                "avg_launch_us": round(avg_us, 3), "launches": nl,
                "bytes_per_launch": round(by / max(nl, 1), 1)}
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
    kernels = {prec: {k: {"ms": round(v[0] / args.steps, 3),
                          "launches": v[1] // args.steps,
                          "avg_us": round(1e3 * v[0] / v[1], 3) if v[1] else 0.0,
                          "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 2) if v[0] > 0 else 0.0}
                      for k, v in acc[prec].items()}
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
        "rel_res": {"fp64": i64["res"] / i64["norm_F"], "mixed": i32["res"] / i32["norm_F"]},
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
        out["cpu_baseline"] = {"value": round(cpu_ms, 1), "unit": "ms", "cores": 1,
                               "kind": "oracle",
                               "sample": "one FP64 solve of the same problem to the same "
                                         "tolerance (plain C oracle, single thread, %d "
                                         "iterations)" % info_o.iterations}
        out["err_vs_oracle"] = {
            "fp64": float(np.abs(U64.cpu().numpy() - ut).max() / scale),
            "mixed": float(np.abs(U32.cpu().numpy() - ut).max() / scale),
            "reference": "oracle FGMRES to scaled relative residual 1e-10, max-norm relative"}
    print(json.dumps(out), flush=True)


def roofline_of(kt, names=None, prefer=None):
    """Roofline entry of the dominant kernel class (or `prefer`) of a timing
    dictionary {class: (ms, launches, algorithmic bytes)}."""
    dom = prefer or max(kt, key=lambda k: kt[k][0])
    ms, nl, by = kt[dom]
    avg_us = 1e3 * ms / max(nl, 1)
    achieved = (by / max(nl, 1)) / (avg_us * 1e-6) / 1e9 if nl else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": (names or {}).get(dom, dom), "avg_launch_us": round(avg_us, 3),
            "launches": nl, "bytes_per_launch": round(by / max(nl, 1), 1)}


def kernels_of(kt, steps):
    return {k: {"ms": round(v[0] / steps, 3), "launches": v[1] // steps,
                "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 2) if v[0] > 0 else 0.0}
            for k, v in kt.items()}


def oracle_pool(jobs):
    """Run oracle solves (callables) one per host core; returns (wall s, cores)."""
    from concurrent.futures import ThreadPoolExecutor
    cores = min(len(jobs), os.cpu_count() or 1)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(lambda f: f(), jobs))
    return time.perf_counter() - t0, cores


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
    for _ in range(args.warmup):
        b.solve(F, **opts)
    a, c = ev(), ev()
    a.record()
    for _ in range(args.steps):
        U, info = b.solve(F, **opts)
    c.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(c) / args.steps
    b.timing(True)
    b.solve(F, **opts)
    kt = b.timing(False)
    it = [d["iterations"] for d in info]
    out = {"metric": "batched solves/s, 64 uneven instances (N in {128..1024}, eps in [1e-8,1e-2]), "
                     "mixed, rel-res 1e-8",
           "value": round(64e3 / ms, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
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
        # bounded sample: the first eight instances with N <= 256 (a full
        # N = 1024 oracle solve can take tens of seconds)
        sample = [i for i in insts if i.N <= 256][:8]

        def job(i):
            def run():
                op = O.Problem(i.N, i.eps, c1=i.c1_at, c2=i.c2_at, r=i.r_const)
                op.fgmres(O.sine_series(i.N, op.x, op.y, i.a), tol=1e-8, scaled=True, maxit=2000)
            return run
        wall, cores = oracle_pool([job(i) for i in sample])
        out["cpu_baseline"] = {"value": round(len(sample) / wall, 3), "unit": "solves/s",
                               "cores": cores, "kind": "oracle",
                               "sample": "the first %d instances with N <= 256 (N %s), one FP64 "
                                         "oracle solve per core; the GPU batch also holds the "
                                         "N = 512 and 1024 instances" % (len(sample),
                                                                         [i.N for i in sample])}
    print(json.dumps(out), flush=True)


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
        return i1, i2
    for _ in range(args.warmup):
        step()
    a, c = ev(), ev()
    a.record()
    for _ in range(args.steps):
        i1, i2 = step()
    c.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(c) / args.steps
    b.timing(True)
    step()
    kt = b.timing(False)
    out = {"metric": "16 right-hand sides at N=2048, eps=1e-6: mixed solves + adjoint gradients",
           "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "N=2048 (4.19M unknowns), eps=1e-6, c=(1+x^2,1+y), r=1, 16 "
                                  "seeded 3x3 sine right-hand sides; 16 FGMRES(50) mixed solves "
                                  "to 1e-8 and 16 adjoint solves, one batch (graphs, autotuned)"},
           "iterations": {"forward": [d["iterations"] for d in i1],
                          "adjoint": [d["iterations"] for d in i2]},
           "setup_s": round(setup_s, 3),
           "footprint_bytes": {"batch": b.footprint(), "problem": p.footprint()},
           "roofline": {"spmv": roofline_of(kt, prefer="spmv"),
                        "sweep": roofline_of(kt, prefer="sweep"),
                        "lines": roofline_of(kt, prefer="lines"),
                        "dominant": roofline_of(kt)},
           "kernels_per_step": kernels_of(kt, 1), "tuning": b.describe()}
    if not args.no_cpu:
        from oracle import oracle as O
        op = O.Problem(inst.N, inst.eps, c1=inst.c1_at, c2=inst.c2_at, r=inst.r_const)
        Fo = O.sine_series(inst.N, op.x, op.y, A[0])
        t1 = time.perf_counter()
        _, _, info_o, _ = op.fgmres(Fo, tol=1e-8, scaled=True, maxit=2000)
        cpu_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(1e3 * cpu_s * 2 * len(F), 1), "unit": "ms",
                               "cores": 1, "kind": "oracle",
                               "sample": "one FP64 oracle solve of the first right-hand side "
                                         "(%d iterations, %.1f s), scaled to 16 forward and 16 "
                                         "adjoint solves" % (info_o.iterations, cpu_s)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--N", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=("headline", "batch", "multi_rhs", "copy_probe"),
                    default="headline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (instances and "
              "right-hand sides shard without communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    {"headline": headline, "batch": batch, "multi_rhs": multi_rhs,
     "copy_probe": copy_probe}[args.workload](args)


if __name__ == "__main__":
    main()
