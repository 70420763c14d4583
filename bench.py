"""Benchmark: grid points hierarchized per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]
                    [--no-cpu-baseline] [--no-extras] [--workload NAME]

One step is one in-place hierarchization (all axes) of the d=3 anisotropic
grid of level (10, 9, 8): 1023 x 511 x 255 = 133,302,015 points, 1.07 GB in
FP64, values prod_k sin(pi x_k) + 0.01 N(0,1) (seed 1), already resident in
HBM.  The step is timed with HIP events on the launch stream; every library
kernel is also bracketed by its own events (sgh_timing_*), which gives the
per-kernel durations behind the roofline figure.

With --workload NAME it times one secondary workload instead and prints its
own JSON line (value, roofline of its dominant kernel, CPU oracle sample):
pole27 (one pole of level 27, 1.07 GB FP64), tend12 (the 10-dimensional
shape (12,2,...,2), 645 MB FP64), combi_d4n15 (gather / scatter between the
d=4, n=15 combination set and its sparse grid, 1.1 GB FP64), batch (the
d=4, n=10 set as one plan) and batch128 (128 copies of that set, 1.0 GB).

Prints one JSON line.  `value` is points/s of the whole job (one GPU).
Extra fields: the inverse and the transpose on the same grid, the batched
combination-technique set (589 grids, one launch) versus a loop of per-grid
calls, the sparse grid of that set (gather, scatter, reduce step) and the
gather / scatter bandwidth on the d=4, n=15 set, a measured copy roof, the
roofline of the dominant kernel and the CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "grid points hierarchized/s + achieved HBM GB/s vs peak; batched vs per-grid speedup"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the schedule of the grid first (timed trial launches on scratch grids)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only copy a buffer of the workload's size (reference kernel for HBM counters)")
    ap.add_argument("--workload", choices=["aniso3d"] + sorted(SECONDARY), default="aniso3d",
                    help="aniso3d (default): the benchmark grid; the others time one secondary workload "
                         "(its own JSON line, roofline of its dominant kernel)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1309_0392_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".inc", ".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str = "aniso3d"):
    """HBM bytes per launch of `kernel` in `workload` from the committed counter
    summary, if it was taken with the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    entry = data.get("workloads", {}).get(workload, {}).get(kernel)
    return None if entry is None else entry.get("bytes_per_launch")


def time_region(torch, fn, steps):
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(s)
    for _ in range(steps):
        fn()
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


# ----------------------------------------------------------- secondary workloads
def timed_kernels(torch, sgh, fn, steps):
    """ms per call of fn over `steps` calls, and the library's per-kernel report."""
    fn()
    torch.cuda.synchronize()
    sgh.timing_reset()
    sgh.timing_enable(True)
    ms = time_region(torch, fn, steps) / steps
    report = sgh.timing_report()
    sgh.timing_enable(False)
    return ms, report


def roofline_of(report, bytes_per_launch, workload, dominant=None):
    """Roofline entry for the kernel with the largest share of the timed region
    (or the named one); bytes_per_launch maps kernel name -> algorithmic bytes."""
    name = dominant or max(report.items(), key=lambda kv: kv[1]["ms"])[0]
    st = report[name]
    avg = st["ms"] / st["count"]
    algo = bytes_per_launch(name)
    ach = algo / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(name, workload), "algorithmic_bytes_per_launch": algo,
            "avg_launch_ms": avg}


def kernel_table(report):
    return {k: {"launches": v["count"], "avg_ms": v["ms"] / v["count"]} for k, v in report.items()}


def secondary_grid(args, torch, np, sgh, W, name):
    """One large grid: the level-27 pole or the 10-dimensional shape (FP64)."""
    if name == "pole27":
        levels, desc = (27,), "one pole of level 27: 134,217,727 points, 1.07 GB FP64"
    else:
        levels, desc = (12,) + (2,) * 9, "10-d (12,2,2,2,2,2,2,2,2,2): 4095 x 3^9 = 80,601,885 points, 645 MB FP64"
    x_host = W.sine_plus_noise(levels, seed=8) if name == "pole27" else W.uniform(levels, 9)
    x = torch.from_numpy(x_host).cuda()
    N = x.numel()
    out = {"metric": "grid points hierarchized/s (%s)" % name, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": desc, "levels": list(levels), "points": N}}
    for _ in range(args.warmup):
        sgh.hierarchize(x, levels)
    ms, rep = timed_kernels(torch, sgh, lambda: sgh.hierarchize(x, levels), args.steps)
    out.update({"value": N / (ms * 1e-3), "ms_per_step": ms, "kernels": kernel_table(rep),
                "schedule": sgh.schedule(sgh.OP_HIERARCHIZE, levels)["launches"],
                "roofline": roofline_of(rep, lambda k: 2.0 * N * 8, name)})
    if not args.no_extras:
        extras = {}
        for nm, op in (("dehierarchize", sgh.OP_DEHIERARCHIZE), ("adjoint", sgh.OP_ADJOINT)):
            ms_o, rep_o = timed_kernels(torch, sgh, lambda op=op: sgh.transform(op, x, levels), args.steps)
            extras[nm] = {"points_per_s": N / (ms_o * 1e-3), "ms": ms_o, "kernels": kernel_table(rep_o)}
        out["extras"] = extras
    if not args.no_cpu_baseline:
        import oracle
        t = time.time()
        oracle.hierarchize(x_host, levels)
        sec = time.time() - t
        out["cpu_baseline"] = {"value": N / sec, "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": "the whole grid, FP64, hierarchized once by the C oracle (one thread)"}
    return out


def secondary_combination(args, torch, np, sgh, W, name):
    """Sparse grid of the d=4, n=15 combination set: gather and scatter (FP64)."""
    lv, co = W.combination_set(4, 15)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(10)
    xs = [torch.rand(W.shape_of(l), dtype=torch.float64, device="cuda", generator=gen) for l in lv]
    npts = sum(t.numel() for t in xs)
    comb = sgh.Combination(xs, lv, co, graph=False)
    sp = comb.new_sparse()
    algo = (npts + comb.sparse_points) * 8.0
    for _ in range(args.warmup):
        comb.gather(sp)
        comb.scatter(sp)
    ms_g, rep_g = timed_kernels(torch, sgh, lambda: comb.gather(sp), args.steps)
    ms_s, rep_s = timed_kernels(torch, sgh, lambda: comb.scatter(sp), args.steps)
    out = {"metric": "grid points gathered into the sparse grid/s (d=4, n=15 combination set)", "unit": "points/s",
           "value": npts / (ms_g * 1e-3), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_g, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "sparse grid of the d=4, n=15 combination set: %d grids, %d grid points, "
                                  "%d sparse points, FP64" % (len(lv), npts, comb.sparse_points)},
           "roofline": roofline_of(rep_g, lambda k: algo, name),
           "extras": {"scatter": {"points_per_s": npts / (ms_s * 1e-3), "ms": ms_s,
                                  "roofline": roofline_of(rep_s, lambda k: algo, name)}}}
    comb.close()
    if not args.no_cpu_baseline:
        import oracle
        lv10, c10 = W.combination_set()
        hs = W.combination_values(lv10, seed=3)
        t = time.time()
        oracle.combi_gather(hs, lv10, c10)
        sec = time.time() - t
        out["cpu_baseline"] = {"value": sum(h.size for h in hs) / sec, "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": "the oracle's gather on the d=4, n=10 set (980,797 grid points), once"}
    return out


def secondary_batch(args, torch, np, sgh, W, name):
    """The d=4, n=10 combination set as one batched plan; `batch128` holds 128 copies
    of the set (75,392 grids, 1.0 GB FP64) so that HBM, not latency, bounds it;
    `batch_d4n13` is the d=4, n=13 set (1,325 grids, 165 MB FP64), whose grids above
    the LDS tile go to the medium launch."""
    if name == "batch_d4n13":
        return secondary_medium(args, torch, np, sgh, W, name)
    lv, co = W.combination_set()
    R = 128 if name == "batch128" else 1
    xs = [torch.from_numpy(a).cuda() for _ in range(R) for a in W.combination_values(lv, seed=3)]
    lvs = [l for _ in range(R) for l in lv]
    npts = sum(t.numel() for t in xs)
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, xs, lvs, graph=True, autotune=True)
    for _ in range(args.warmup):
        plan.execute()
    ms, rep = timed_kernels(torch, sgh, plan.execute, args.steps)
    out = {"metric": "grid points hierarchized/s (batched combination set)", "unit": "points/s",
           "value": npts / (ms * 1e-3), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "%d copies of the d=4, n=10 combination set: %d grids, %d points, FP64"
                                  % (R, len(lvs), npts)},
           "kernels": kernel_table(rep), "plan": plan.describe()["batches"],
           "roofline": roofline_of(rep, lambda k: 2.0 * npts * 8, name)}
    plan.close()
    return out


def secondary_medium(args, torch, np, sgh, W, name):
    """The d=4, n=13 combination set as one plan: a batch launch for the grids that fit
    the LDS tile and a medium launch (one workgroup per grid, passes through its tile)."""
    lv, _ = W.combination_set(4, 13)
    xs = [torch.from_numpy(a).cuda() for a in W.combination_values(lv, seed=3)]
    npts = sum(t.numel() for t in xs)
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, xs, lv, graph=False)  # two launches, timed one by one
    desc = plan.describe()
    pts = {"hier_f64_batch": sum(b["points"] for b in desc["batches"]),
           "hier_f64_medium": sum(m["points"] for m in desc["medium"])}
    for _ in range(args.warmup):
        plan.execute()
    ms, rep = timed_kernels(torch, sgh, plan.execute, args.steps)
    out = {"metric": "grid points hierarchized/s (batched combination set)", "unit": "points/s",
           "value": npts / (ms * 1e-3), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "the d=4, n=13 combination set: %d grids, %d points (%d in medium grids), FP64"
                                  % (len(lv), npts, pts["hier_f64_medium"])},
           "kernels": kernel_table(rep), "plan": {"batches": desc["batches"], "medium": desc["medium"]},
           "roofline": roofline_of(rep, lambda k: 2.0 * pts.get(k, npts) * 8, name, dominant="hier_f64_medium")}
    plan.close()
    return out


SECONDARY = {"pole27": secondary_grid, "tend12": secondary_grid, "combi_d4n15": secondary_combination,
             "batch": secondary_batch, "batch128": secondary_batch, "batch_d4n13": secondary_batch}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform of one grid, or of a combination set, "
              "runs on a single device here (multi-GPU sharding is described in DESIGN.md, not built); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1309_0392_amd import sgh
    from paper_1309_0392_amd import workloads as W

    sgh.lib()  # fails loudly if the HIP library is not built
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload != "aniso3d":
        print(json.dumps(SECONDARY[args.workload](args, torch, np, sgh, W, args.workload)))
        return
    dt_np = np.float64 if args.dtype == "f64" else np.float32
    esize = 8 if args.dtype == "f64" else 4
    levels = W.ANISO_3D
    N = W.num_points(levels)

    if args.copy_only:
        a = torch.empty(N, dtype=torch.float64 if esize == 8 else torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        ms = time_region(torch, lambda: b.copy_(a), 10) / 10
        print(json.dumps({"copy_bytes_read": N * esize, "copy_bytes_written": N * esize, "copies": 10,
                          "copy_GBps": 2.0 * N * esize / (ms * 1e-3) / 1e9}))
        return

    t0 = time.time()
    x_host = W.sine_plus_noise(levels, seed=1).astype(dt_np, copy=False)
    x = torch.from_numpy(x_host).to(dev)
    torch.cuda.synchronize()
    gen_s = time.time() - t0

    tuned = {}
    if args.autotune:
        # time the candidate schedules on scratch grids of the same shape; the
        # one-shot calls below then use the chosen schedule (kept in-process)
        for op in (sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT):
            plan = sgh.Plan(op, [x], [levels], graph=False, autotune=True)
            tuned[op] = plan.describe()["large"][0]["launches"]
            plan.close()

    step = lambda: sgh.hierarchize(x, levels)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    sgh.timing_reset()
    sgh.timing_enable(True)
    ms_total = time_region(torch, step, args.steps)
    report = sgh.timing_report()
    sgh.timing_enable(False)
    ms_per_step = ms_total / args.steps
    value = N / (ms_per_step * 1e-3)

    # dominant kernel: the one with the largest share of the timed region
    dom = max(report.items(), key=lambda kv: kv[1]["ms"])
    dom_name, dom_stats = dom[0], dom[1]
    dom_ms = dom_stats["ms"] / dom_stats["count"]
    algo_bytes = 2.0 * N * esize  # each launch reads and writes every point once
    achieved = algo_bytes / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom_name)
    kernels = {k: {"launches": v["count"], "avg_ms": v["ms"] / v["count"],
                   "GBps_algorithmic": algo_bytes / (v["ms"] / v["count"] * 1e-3) / 1e9}
               for k, v in report.items()}
    launches_per_step = sum(v["count"] for v in report.values()) / args.steps
    whole_GBps = 2.0 * N * esize / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "hierarchize d=3 level (10,9,8): 1023x511x255 = %d points, %s, "
                               "prod sin(pi x_k) + 0.01 N(0,1), seed 1" % (N, args.dtype.upper()),
                   "levels": list(levels), "points": N, "bytes": N * esize},
        "hbm_GBps_one_round_trip": whole_GBps,
        "hbm_frac_of_peak_one_round_trip": whole_GBps / HBM_PEAK_GBS,
        "launches_per_step": launches_per_step,
        "schedule": tuned.get(sgh.OP_HIERARCHIZE) or sgh.schedule(sgh.OP_HIERARCHIZE, levels,
                                                                   sgh.F64 if esize == 8 else sgh.F32)["launches"],
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": algo_bytes,
                     "avg_launch_ms": dom_ms},
    }

    if not args.no_extras:
        extras = {}
        # inverse and transpose on the same grid
        for name, op in (("dehierarchize", sgh.OP_DEHIERARCHIZE), ("adjoint", sgh.OP_ADJOINT)):
            f = lambda op=op: sgh.transform(op, x, levels)
            f()
            ms = time_region(torch, f, max(3, args.steps // 2)) / max(3, args.steps // 2)
            extras[name + "_points_per_s"] = N / (ms * 1e-3)
        # measured copy roof on the same bytes
        y = torch.empty_like(x)
        y.copy_(x)
        ms = time_region(torch, lambda: y.copy_(x), 10) / 10
        extras["copy_GBps"] = 2.0 * N * esize / (ms * 1e-3) / 1e9
        del y
        # batched combination technique set vs per-grid calls
        lv, _ = W.combination_set()
        for bdt, bname in ((np.float64, "f64"), (np.float32, "f32")):
            xs = [torch.from_numpy(a).to(dev) for a in W.combination_values(lv, seed=3, dtype=bdt)]
            npts = sum(t.numel() for t in xs)
            plan = sgh.Plan(sgh.OP_HIERARCHIZE, xs, lv, graph=True, autotune=True)
            plan.execute()
            ms_plan = time_region(torch, plan.execute, 50) / 50

            def loop():
                for t, l in zip(xs, lv):
                    sgh.hierarchize(t, l)
            loop()
            ms_loop = time_region(torch, loop, 5) / 5
            extras["batch_" + bname] = {"grids": len(lv), "points": npts, "plan_ms": ms_plan,
                                        "points_per_s": npts / (ms_plan * 1e-3),
                                        "per_grid_loop_ms": ms_loop, "speedup_vs_per_grid": ms_loop / ms_plan,
                                        "plan": plan.describe()["batches"]}
            plan.close()
        # combination technique: sparse grid of the d=4, n=10 set (gather, scatter,
        # and the solver-free reduce step hierarchize -> gather -> scatter -> dehierarchize)
        xs = [torch.from_numpy(a).to(dev) for a in W.combination_values(lv, seed=3)]
        npts = sum(t.numel() for t in xs)
        comb = sgh.Combination(xs, lv, W.combination_set()[1], graph=True)
        sp = comb.new_sparse()
        ms_g = time_region(torch, lambda: comb.gather(sp), 50) / 50
        ms_s = time_region(torch, lambda: comb.scatter(sp), 50) / 50
        ms_r = time_region(torch, lambda: comb.reduce(sp), 20) / 20
        extras["combination_d4n10_f64"] = {
            "grids": len(lv), "grid_points": npts, "sparse_points": comb.sparse_points,
            "gather_ms": ms_g, "scatter_ms": ms_s, "reduce_ms": ms_r,
            "reduce_grid_points_per_s": npts / (ms_r * 1e-3)}
        comb.close()
        del xs, sp
        # the same on the d=4, n=15 set (2059 grids, 1.1 GB FP64): gather / scatter bandwidth
        lv15, c15 = W.combination_set(4, 15)
        gen = torch.Generator(device=dev)
        gen.manual_seed(5)
        xs = [torch.rand(W.shape_of(l), dtype=torch.float64, device=dev, generator=gen) for l in lv15]
        npts = sum(t.numel() for t in xs)
        comb = sgh.Combination(xs, lv15, c15, graph=False)
        sp = comb.new_sparse()
        ms_g = time_region(torch, lambda: comb.gather(sp), 10) / 10
        ms_s = time_region(torch, lambda: comb.scatter(sp), 10) / 10
        algo = (npts + comb.sparse_points) * 8.0  # every grid point read or written once, sparse once
        extras["combination_d4n15_f64"] = {
            "grids": len(lv15), "grid_points": npts, "sparse_points": comb.sparse_points,
            "gather_ms": ms_g, "scatter_ms": ms_s,
            "gather_GBps_algorithmic": algo / (ms_g * 1e-3) / 1e9,
            "scatter_GBps_algorithmic": algo / (ms_s * 1e-3) / 1e9}
        comb.close()
        del xs, sp
        out["extras"] = extras

    if not args.no_cpu_baseline:
        import oracle
        reps = 3
        times = []
        for _ in range(reps):
            t = time.time()
            oracle.hierarchize(x_host.astype(np.float64, copy=False), levels)
            times.append(time.time() - t)
        med = sorted(times)[reps // 2]
        out["cpu_baseline"] = {"value": N / med, "unit": "points/s", "cores": 1, "kind": "oracle",
                               "sample": "the full (10,9,8) grid, FP64, hierarchized by the C oracle "
                                         "(Algorithm 1, single thread) %d times, median; includes the "
                                         "oracle's input copy" % reps}
    out["input_generation_s"] = gen_s
    print(json.dumps(out))


if __name__ == "__main__":
    main()
