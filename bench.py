"""Benchmark: grid points hierarchized per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32]
                    [--no-cpu-baseline] [--no-extras] [--workload NAME]

One step is one in-place hierarchization (all axes) of the d=3 anisotropic
grid of level (10, 9, 8): 1023 x 511 x 255 = 133,302,015 points, 1.07 GB in
FP64, values prod_k sin(pi x_k) + 0.01 N(0,1) (seed 1), already resident in
HBM.  K steps run back to back between two stream synchronizations and are
timed with HIP events on the launch stream; every library kernel is also
bracketed by its own events (sgh_timing_*), which gives the per-kernel
durations behind the roofline figure.  A second protocol alternates
hierarchization and dehierarchization (each call timed on its own, warm, then
cold after a 512 MB write that evicts the caches) and reports median and
minimum.

With --workload NAME it times another workload and prints its own JSON line
(value, roofline of its dominant kernel, CPU oracle sample):
  aniso5d      the 5-d grid (6,6,5,5,5), 0.95 GB FP64, values U[-1,1] (seed 2)
  pole27       one pole of level 27, 1.07 GB FP64
  tend12       the 10-d shape (12,2,...,2), 645 MB FP64
  combi_d4n15  gather / scatter between the d=4, n=15 set and its sparse grid
  batch        the d=4, n=10 combination set (589 grids) as one plan, with the
               per-grid baselines (one C call for all grids; a Python loop)
  batch128     128 copies of that set in one plan (1.0 GB FP64)
  batch_d4n13  the d=4, n=13 set (1,325 grids, 165 MB FP64)
  grad_d4n10   forward + backward of loss = sum_l c_l ||H u_l||^2 over the
               d=4, n=10 set in FP32 through torch.autograd (the set stored back
               to back in one tensor); --replicas R takes R copies of the set
`--dtype` selects FP64 or FP32 storage for every transform workload.

Prints one JSON line.  `value` is points/s of the whole job (one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "grid points hierarchized/s + achieved HBM GB/s vs peak; batched vs per-grid speedup"
FLUSH_BYTES = 512 << 20  # cold reps: write this much between calls (the Infinity Cache is 256 MB)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f64", "f32"], default=None,
                    help="storage type (default f64; f32 for grad_d4n10)")
    ap.add_argument("--replicas", type=int, default=1, help="grad_d4n10: copies of the set")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the schedule of the grid first (timed trial launches on scratch grids)")
    ap.add_argument("--copy-only", action="store_true",
                    help="only copy a buffer of the workload's size (reference kernel for HBM counters)")
    ap.add_argument("--out-of-place", action="store_true",
                    help="single grids: the timed step transforms into a second resident buffer (sgh_transform_out)")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the warm-up and the timed steps (no protocol, extras or CPU baseline): for profilers")
    ap.add_argument("--op", choices=["hierarchize", "dehierarchize", "adjoint"], default="hierarchize",
                    help="single grids, in place: the operation of the timed steps (default hierarchize)")
    ap.add_argument("--workload", choices=sorted(GRIDS) + sorted(SECONDARY), default="aniso3d")
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


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


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


def stats(ms):
    ms = sorted(ms)
    return {"median_ms": ms[len(ms) // 2], "min_ms": ms[0], "max_ms": ms[-1], "reps": len(ms)}


def protocol(torch, fwd, inv, reps=20, cold=5):
    """Alternate fwd and inv (each call timed on its own with events on the
    stream), then `cold` fwd calls each after a 512 MB write; median and min."""
    s = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for _ in range(3):  # warm-up
        fwd()
        inv()
    marks = []
    torch.cuda.synchronize()
    for _ in range(reps):
        for which, fn in (("f", fwd), ("i", inv)):
            a, b = ev(), ev()
            a.record(s)
            fn()
            b.record(s)
            marks.append((which, a, b))
    flush = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
    for r in range(cold):
        flush.fill_(float(r))
        a, b = ev(), ev()
        a.record(s)
        fwd()
        b.record(s)
        marks.append(("c", a, b))
        inv()
    torch.cuda.synchronize()
    out = {}
    for key, name in (("f", "forward"), ("i", "inverse"), ("c", "forward_cold")):
        out[name] = stats([a.elapsed_time(b) for w, a, b in marks if w == key])
    del flush
    return out


def timed_kernels(torch, sgh, fn, steps, separate=False):
    """ms per call of fn over `steps` calls, and the library's per-kernel report
    (HIP events around every launch, on its stream, over the same timed calls).
    separate=True (workloads of a few microseconds, where the events' own cost
    would show in the step time): the steps are timed without the per-launch
    events, and the report comes from as many calls right after."""
    fn()
    torch.cuda.synchronize()
    if separate:
        ms = time_region(torch, fn, steps) / steps
    sgh.timing_reset()
    sgh.timing_enable(True)
    ms_inst = time_region(torch, fn, steps) / steps
    report = sgh.timing_report()
    sgh.timing_enable(False)
    return (ms if separate else ms_inst), report


def roofline_of(report, bytes_per_launch, workload, dominant=None):
    """Roofline entry for the kernel with the largest share of the timed region
    (or the named one); bytes_per_launch maps kernel name -> algorithmic bytes."""
    name = dominant or max(report.items(), key=lambda kv: kv[1]["ms"])[0]
    st = report[name]
    avg = st["ms"] / st["count"]
    algo = bytes_per_launch(name)
    ach = algo / (avg * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(name, workload),
            "algorithmic_bytes_per_launch": algo, "avg_launch_ms": avg}


def kernel_table(report, algo_bytes=None):
    out = {}
    for k, v in report.items():
        avg = v["ms"] / v["count"]
        out[k] = {"launches": v["count"], "avg_ms": avg}
        if algo_bytes:
            b = algo_bytes(k)
            if b:
                out[k]["GBps_algorithmic"] = b / (avg * 1e-3) / 1e9
    return out


def cpu_oracle_timing(run, reps_single, reps_threads, sample, unit_count, unit="points/s"):
    """The oracle as it stands, on one thread and on every core (OpenMP over
    poles), `run(threads)` timed `reps` times each; median."""
    import oracle
    out = {}
    for threads, reps in ((False, reps_single), (True, reps_threads)):
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            run(threads)
            times.append(time.perf_counter() - t)
        med = sorted(times)[len(times) // 2]
        out["threads" if threads else "single"] = {"value": unit_count / med, "seconds": med, "reps": reps,
                                                   "cores": oracle.num_threads(threads)}
    best = out["threads"]
    res = {"value": best["value"], "unit": unit, "cores": best["cores"], "kind": "oracle",
           "sample": sample + "; value: all cores (OpenMP over the poles of each direction), "
                              "single_thread beside it; median of the reps",
           "single_thread": out["single"], "all_cores": out["threads"]}
    res.update(host_info())
    return res


def dtype_of(args, default="f64"):
    return args.dtype or default


# ------------------------------------------------------------- single grids
GRIDS = {
    "aniso3d": "hierarchize d=3 level (10,9,8): 1023x511x255 = {N} points, {DT}, prod sin(pi x_k) + 0.01 N(0,1), "
               "seed 1",
    "aniso5d": "hierarchize d=5 level (6,6,5,5,5): 63x63x31x31x31 = {N} points, {DT}, U[-1,1], seed 2",
    "pole27": "hierarchize one pole of level 27: {N} points, {DT}, sine + noise, seed 8",
    "tend12": "hierarchize the 10-d shape (12,2,2,2,2,2,2,2,2,2): 4095 x 3^9 = {N} points, {DT}, U[-1,1], seed 9",
}


def grid_input(W, name):
    if name == "aniso3d":
        return W.ANISO_3D, W.sine_plus_noise(W.ANISO_3D, seed=1)
    if name == "aniso5d":
        return W.ANISO_5D, W.uniform(W.ANISO_5D, seed=2)
    if name == "pole27":
        return (27,), W.sine_plus_noise((27,), seed=8)
    levels = (12,) + (2,) * 9
    return levels, W.uniform(levels, 9)


def run_grid(args, torch, np, sgh, W, name):
    dt = dtype_of(args)
    esize = 8 if dt == "f64" else 4
    t0 = time.time()
    levels, x_host = grid_input(W, name)
    x_host = x_host.astype(np.float64 if dt == "f64" else np.float32, copy=False)
    x = torch.from_numpy(x_host).cuda()
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    N = x.numel()
    code = sgh.F64 if dt == "f64" else sgh.F32

    if args.copy_only:
        b = torch.empty_like(x)
        ms = time_region(torch, lambda: b.copy_(x), 10) / 10
        return {"copy_bytes_read": N * esize, "copy_bytes_written": N * esize, "copies": 10,
                "copy_GBps": 2.0 * N * esize / (ms * 1e-3) / 1e9}

    tuned = {}
    if args.autotune:
        for op in (sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT):
            plan = sgh.Plan(op, [x], [levels], graph=False, autotune=True)
            tuned[op] = plan.describe()["large"][0]["launches"]
            plan.close()

    step_op = {"hierarchize": sgh.OP_HIERARCHIZE, "dehierarchize": sgh.OP_DEHIERARCHIZE,
               "adjoint": sgh.OP_ADJOINT}[args.op]
    if step_op != sgh.OP_HIERARCHIZE and (args.out_of_place or args.autotune):
        raise SystemExit("--op other than hierarchize: in place and with the default schedule only")
    if args.out_of_place:
        y_out = torch.empty_like(x)
        step = lambda: sgh.transform_out(sgh.OP_HIERARCHIZE, x, y_out, levels)
    elif step_op != sgh.OP_HIERARCHIZE:
        step = lambda: sgh.transform(step_op, x, levels)
    else:
        step = lambda: sgh.hierarchize(x, levels)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    algo = 2.0 * N * esize  # each transform launch reads and writes every point once
    sgh.timing_reset()
    sgh.timing_enable(True)
    ms_total = time_region(torch, step, args.steps)
    report = sgh.timing_report()
    sgh.timing_enable(False)
    ms = ms_total / args.steps
    sched = tuned.get(sgh.OP_HIERARCHIZE) or sgh.schedule(step_op, levels, code,
                                                           out_of_place=args.out_of_place)["launches"]
    whole = algo / (ms * 1e-3) / 1e9
    wl = (name if dt == "f64" else name + "_f32") + ("_out" if args.out_of_place else "")
    if step_op != sgh.OP_HIERARCHIZE:
        wl += "_" + args.op
    if step_op == sgh.OP_HIERARCHIZE:
        metric = METRIC if name == "aniso3d" else "grid points hierarchized/s (%s)" % name
    else:
        metric = "grid points %s/s (%s)" % ("dehierarchized" if step_op == sgh.OP_DEHIERARCHIZE else
                                              "transformed by the adjoint", name)
    out = {
        "metric": metric,
        "value": N / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
        "data": "synthetic",
        "config": {"workload": GRIDS[name].format(N=N, DT=dt.upper()), "levels": list(levels), "points": N,
                   "bytes": N * esize},
        "hbm_GBps_one_round_trip": whole, "hbm_frac_of_peak_one_round_trip": whole / HBM_PEAK_GBS,
        "launches_per_step": sum(v["count"] for v in report.values()) / args.steps,
        "schedule": sched,
        "kernels": kernel_table(report, lambda k: algo),
        "roofline": roofline_of(report, lambda k: algo, wl),
    }
    if args.out_of_place:
        out["config"]["workload"] += ", out of place into a second resident buffer"
    if step_op != sgh.OP_HIERARCHIZE:
        out["config"]["workload"] += ", operation: " + args.op
    if args.profile_run or step_op != sgh.OP_HIERARCHIZE:
        return out
    out["timing_protocol"] = protocol(torch, step, lambda: sgh.dehierarchize(x, levels))
    out["timing_protocol"]["points_per_s_median"] = N / (out["timing_protocol"]["forward"]["median_ms"] * 1e-3)
    out["out_of_place"] = out_of_place(args, torch, sgh, x, levels, code, algo, name if dt == "f64" else name + "_f32")

    if not args.no_extras:
        extras = {}
        for nm, op in (("dehierarchize", sgh.OP_DEHIERARCHIZE), ("adjoint", sgh.OP_ADJOINT)):
            f = lambda op=op: sgh.transform(op, x, levels)
            ms_o, rep_o = timed_kernels(torch, sgh, f, max(3, args.steps // 2))
            extras[nm] = {"points_per_s": N / (ms_o * 1e-3), "ms": ms_o, "kernels": kernel_table(rep_o, lambda k: algo),
                          "schedule": sgh.schedule(op, levels, code)["launches"]}
        y = torch.empty_like(x)
        y.copy_(x)
        ms_c = time_region(torch, lambda: y.copy_(x), 10) / 10
        extras["copy_GBps"] = 2.0 * N * esize / (ms_c * 1e-3) / 1e9
        del y
        if name == "aniso3d":
            extras.update(batch_extras(torch, np, sgh, W))
        out["extras"] = extras

    if not args.no_cpu_baseline:
        import oracle
        x64 = np.ascontiguousarray(x_host, dtype=np.float64)
        work = np.empty_like(x64)

        def run(threads):
            np.copyto(work, x64)
            oracle.hierarchize_inplace(work, levels, threads)
        # the refill of the work array is outside the oracle but inside the timing: subtract it
        t = time.perf_counter()
        for _ in range(3):
            np.copyto(work, x64)
        refill = (time.perf_counter() - t) / 3
        cb = cpu_oracle_timing(run, 3, 10, "the whole grid in FP64 (the FP64 values the GPU run starts from), "
                                           "hierarchized by the C oracle (Algorithm 1, -O2)", N)
        for k in ("single_thread", "all_cores"):
            sec = max(cb[k]["seconds"] - refill, 1e-9)
            cb[k]["seconds"] = sec
            cb[k]["value"] = N / sec
        cb["value"] = cb["all_cores"]["value"]
        out["cpu_baseline"] = cb
        del work, x64
    out["input_generation_s"] = gen_s
    return out


def out_of_place(args, torch, sgh, x, levels, code, algo, workload):
    """The same grid transformed out of place (sgh_transform_out) into a second
    resident buffer: hierarchization (whose fused launch also takes the next
    axis), and the inverse and transpose of the result."""
    N = x.numel()
    y = torch.empty_like(x)
    res = {}
    for nm, op in (("hierarchize", sgh.OP_HIERARCHIZE), ("dehierarchize", sgh.OP_DEHIERARCHIZE),
                   ("adjoint", sgh.OP_ADJOINT)):
        f = lambda op=op: sgh.transform_out(op, x, y, levels)
        for _ in range(args.warmup):
            f()
        ms, rep = timed_kernels(torch, sgh, f, args.steps)
        res[nm] = {"points_per_s": N / (ms * 1e-3), "ms": ms, "kernels": kernel_table(rep, lambda k: algo),
                   "schedule": sgh.schedule(op, levels, code, out_of_place=True)["launches"],
                   "hbm_round_trips": sgh.schedule(op, levels, code, out_of_place=True)["hbm_round_trips"],
                   "roofline": roofline_of(rep, lambda k: algo, workload + "_out")}
    del y
    return res


def batch_extras(torch, np, sgh, W):
    """The d=4, n=10 set (589 grids) as one plan against the per-grid paths,
    and its sparse grid (gather, scatter, reduce); gather / scatter bandwidth on
    the d=4, n=15 set."""
    extras = {}
    lv, co = W.combination_set()
    for bdt, bname in ((np.float64, "f64"), (np.float32, "f32")):
        xs = [torch.from_numpy(a).cuda() for a in W.combination_values(lv, seed=3, dtype=bdt)]
        extras["batch_" + bname] = batch_vs_per_grid(torch, sgh, xs, lv)
    xs = [torch.from_numpy(a).cuda() for a in W.combination_values(lv, seed=3)]
    npts = sum(t.numel() for t in xs)
    comb = sgh.Combination(xs, lv, co, graph=True)
    sp = comb.new_sparse()
    ms_g = time_region(torch, lambda: comb.gather(sp), 50) / 50
    ms_s = time_region(torch, lambda: comb.scatter(sp), 50) / 50
    ms_r = time_region(torch, lambda: comb.reduce(sp), 20) / 20
    extras["combination_d4n10_f64"] = {
        "grids": len(lv), "grid_points": npts, "sparse_points": comb.sparse_points,
        "gather_ms": ms_g, "scatter_ms": ms_s, "reduce_ms": ms_r, "reduce_grid_points_per_s": npts / (ms_r * 1e-3)}
    comb.close()
    del xs, sp
    lv15, c15 = W.combination_set(4, 15)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    xs = [torch.rand(W.shape_of(l), dtype=torch.float64, device="cuda", generator=gen) for l in lv15]
    npts = sum(t.numel() for t in xs)
    comb = sgh.Combination(xs, lv15, c15, graph=False)
    sp = comb.new_sparse()
    ms_g = time_region(torch, lambda: comb.gather(sp), 10) / 10
    ms_s = time_region(torch, lambda: comb.scatter(sp), 10) / 10
    algo = (npts + comb.sparse_points) * 8.0  # every grid point read or written once, sparse once
    extras["combination_d4n15_f64"] = {
        "grids": len(lv15), "grid_points": npts, "sparse_points": comb.sparse_points,
        "gather_ms": ms_g, "scatter_ms": ms_s, "gather_GBps_algorithmic": algo / (ms_g * 1e-3) / 1e9,
        "scatter_GBps_algorithmic": algo / (ms_s * 1e-3) / 1e9}
    comb.close()
    return extras


def batch_vs_per_grid(torch, sgh, xs, lv):
    """One plan (one batched launch) against the library's per-grid path: one C
    call sgh_hierarchize over all grids (the library issues each grid's own
    launches), and a Python loop of one call per grid."""
    npts = sum(t.numel() for t in xs)
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, xs, lv, graph=True, autotune=True)
    plan.execute()
    ms_plan = time_region(torch, plan.execute, 50) / 50
    one_call = lambda: sgh.hierarchize(xs, lv)
    one_call()
    ms_call = time_region(torch, one_call, 10) / 10

    def loop():
        for t, l in zip(xs, lv):
            sgh.hierarchize(t, l)
    loop()
    ms_loop = time_region(torch, loop, 5) / 5
    res = {"grids": len(lv), "points": npts, "plan_ms": ms_plan, "points_per_s": npts / (ms_plan * 1e-3),
           "per_grid_one_call_ms": ms_call, "speedup_vs_per_grid_one_call": ms_call / ms_plan,
           "per_grid_python_loop_ms": ms_loop, "speedup_vs_per_grid_python_loop": ms_loop / ms_plan,
           "plan": plan.describe()["batches"]}
    res["graph_replay"] = graph_replay(torch, plan, xs)
    plan.close()
    return res


def graph_replay(torch, plan, xs):
    """The plan's launch captured once into a graph (torch.cuda.CUDAGraph) and
    replayed, beside the direct launch: each of three replays, with eager work
    and synchronizations between them, must equal a direct execute from the
    same inputs bit for bit before the replays are timed."""
    try:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.execute()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            plan.execute()
        torch.cuda.synchronize()
        for _ in range(3):
            before = [t.clone() for t in xs]
            g.replay()
            torch.cuda.synchronize()
            replayed = [t.clone() for t in xs]
            for t, b in zip(xs, before):
                t.copy_(b)
            plan.execute()
            torch.cuda.synchronize()
            if not all(bool(torch.equal(a, b)) for a, b in zip(replayed, xs)):
                return {"error": "a replay differs from the direct launch"}
        ms = time_region(torch, g.replay, 50) / 50
        del g
        return {"ms": ms, "direct_ms_same_run": time_region(torch, plan.execute, 50) / 50, "replays_checked": 3}
    except Exception as e:  # capture refused by the runtime: report, do not fail the bench
        return {"error": "%s: %s" % (type(e).__name__, e)}


# ------------------------------------------------------- secondary workloads
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
    if not args.no_cpu_baseline and not args.profile_run:
        import oracle
        lv10, c10 = W.combination_set()
        hs = W.combination_values(lv10, seed=3)
        t = time.perf_counter()
        oracle.combi_gather(hs, lv10, c10)
        sec = time.perf_counter() - t
        out["cpu_baseline"] = {"value": sum(h.size for h in hs) / sec, "unit": "points/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "the oracle's gather on the d=4, n=10 set (980,797 grid points), once"}
        out["cpu_baseline"].update(host_info())
    return out


def set_cpu_baseline(np, W, lv, xs64, sample):
    import oracle
    works = [np.empty_like(x) for x in xs64]

    def run(threads):
        for w, x, l in zip(works, xs64, lv):
            np.copyto(w, x)
            oracle.hierarchize_inplace(w, l, threads)
    return cpu_oracle_timing(run, 3, 5, sample, sum(x.size for x in xs64))


def secondary_batch(args, torch, np, sgh, W, name):
    """The d=4, n=10 combination set as one batched plan; `batch128` holds 128
    copies of the set (75,392 grids, 1.0 GB FP64) so that HBM, not latency,
    bounds it; `batch_d4n13` is the d=4, n=13 set (1,325 grids, 165 MB FP64),
    whose grids above the LDS tile go to the medium launch."""
    dt = dtype_of(args)
    npdt = np.float64 if dt == "f64" else np.float32
    esize = 8 if dt == "f64" else 4
    if name == "batch_d4n13":
        lv, _ = W.combination_set(4, 13)
        R = 1
    else:
        lv, _ = W.combination_set()
        R = 128 if name == "batch128" else 1
    host = W.combination_values(lv, seed=3, dtype=npdt)
    xs = [torch.from_numpy(a).cuda() for _ in range(R) for a in host]
    lvs = [l for _ in range(R) for l in lv]
    npts = sum(t.numel() for t in xs)
    # several launches go out directly (not one graph), so that each is timed on its own
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, xs, lvs, graph=False, autotune=(name != "batch_d4n13"))
    desc = plan.describe()
    pts = {}
    for b in desc["batches"]:
        suffix = "_c%dk" % (b["class_bytes"] // 1024) if b["class_bytes"] else ""
        pts["hier_%s_batch%s" % (dt, suffix)] = b["points"]
    for m in desc["medium"]:
        pts["hier_%s_medium" % dt] = m["points"]
    for _ in range(args.warmup):
        plan.execute()
    ms, rep = timed_kernels(torch, sgh, plan.execute, args.steps, separate=(R == 1))
    algo = lambda k: 2.0 * pts.get(k, npts) * esize
    out = {"metric": "grid points hierarchized/s (batched combination set)", "unit": "points/s",
           "value": npts / (ms * 1e-3), "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt, "data": "synthetic",
           "config": {"workload": "%d cop%s of the d=4, n=%d combination set: %d grids, %d points, %s"
                                  % (R, "y" if R == 1 else "ies", 13 if name == "batch_d4n13" else 10, len(lvs),
                                     npts, dt.upper())},
           "kernels": kernel_table(rep, algo), "plan": {"batches": desc["batches"], "medium": desc["medium"]}}
    # the whole execute counts every grid once: its bytes over its time
    whole = 2.0 * npts * esize / (ms * 1e-3) / 1e9
    out["hbm_GBps_whole_plan"] = whole
    out["hbm_frac_of_peak_whole_plan"] = whole / HBM_PEAK_GBS
    dom = "hier_%s_medium" % dt if name == "batch_d4n13" else None
    out["roofline"] = roofline_of(rep, algo, name if dt == "f64" else name + "_f32", dominant=dom)
    plan.close()
    if args.profile_run:
        return out
    if name == "batch" and not args.no_extras:
        out["extras"] = {"per_grid": batch_vs_per_grid(torch, sgh, xs, lvs)}
    if not args.no_cpu_baseline:
        xs64 = [a.astype(np.float64) for a in host]
        out["cpu_baseline"] = set_cpu_baseline(
            np, W, lv, xs64, "one copy of the set (%d grids, %d points), FP64, each grid hierarchized by the C "
                             "oracle" % (len(lv), sum(x.size for x in xs64)))
    return out


def secondary_grad(args, torch, np, sgh, W, name):
    """Forward + backward of loss = sum_l c_l ||H u_l||^2 over the d=4, n=10 set
    (FP32 by default) through torch.autograd: the set lives back to back in one
    tensor; forward and backward are one relative plan each (batched
    hierarchization, batched adjoint), the loss and its gradient torch ops."""
    from paper_1309_0392_amd import autograd as AG
    dt = dtype_of(args, "f32")
    npdt = np.float64 if dt == "f64" else np.float32
    tdt = torch.float64 if dt == "f64" else torch.float32
    esize = 8 if dt == "f64" else 4
    R = max(1, args.replicas)
    lv, co = W.combination_set()
    host = W.combination_values(lv, seed=3, dtype=npdt)
    lvs = [l for _ in range(R) for l in lv]
    flat = np.concatenate([a.ravel() for _ in range(R) for a in host])
    w = np.concatenate([np.full(a.size, c, dtype=npdt) for _ in range(R) for a, c in zip(host, co)])
    u = torch.from_numpy(flat).cuda().requires_grad_(True)
    wt = torch.from_numpy(w).cuda()
    npts = u.numel()
    fs = AG.FlatSet(lvs, tdt)  # plans built once, outside the timed steps

    def step():
        y = fs.hierarchize(u)
        loss = (wt * y * y).sum()
        (g,) = torch.autograd.grad(loss, u)
        return g
    for _ in range(args.warmup):
        step()
    ms, rep = timed_kernels(torch, sgh, step, args.steps, separate=(R == 1))
    pts = {}
    for op, plan in (("hier", fs.fwd), ("adjoint", fs.adj)):
        for b in plan.describe()["batches"]:
            suffix = "_c%dk" % (b["class_bytes"] // 1024) if b["class_bytes"] else ""
            pts["%s_%s_batch%s" % (op, dt, suffix)] = b["points"]
    algo = lambda k: 2.0 * pts.get(k, npts) * esize
    out = {"metric": "grid points differentiated/s (forward + adjoint of the combination-set loss)",
           "unit": "points/s", "value": npts / (ms * 1e-3), "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dt, "data": "synthetic",
           "config": {"workload": "loss sum_l c_l ||H u_l||^2 and its gradient through torch.autograd over %d "
                                  "cop%s of the d=4, n=10 combination set: %d grids, %d points, %s"
                                  % (R, "y" if R == 1 else "ies", len(lvs), npts, dt.upper())},
           "kernels": kernel_table(rep, algo),
           "library_kernel_ms_per_step": sum(v["ms"] for v in rep.values()) / args.steps,
           "roofline": roofline_of(rep, algo, (name if R == 1 else "%s_r%d" % (name, R)) + ("" if dt == "f32" else "_f64"))}
    if not args.no_cpu_baseline and not args.profile_run:
        import oracle
        xs64 = [a.astype(np.float64) for a in host]
        works = [np.empty_like(x) for x in xs64]

        def run(threads):
            for wk, x, l, c in zip(works, xs64, lv, co):
                np.copyto(wk, x)
                oracle.hierarchize_inplace(wk, l, threads)
                wk *= 2.0 * c
                oracle.hierarchize_adjoint_inplace(wk, l, threads)
        out["cpu_baseline"] = cpu_oracle_timing(
            run, 3, 5, "the gradient 2 c_l H^T H u_l of one copy of the set (%d points), FP64, by the C oracle's "
                       "hierarchization and transpose" % sum(x.size for x in xs64), sum(x.size for x in xs64))
    return out


SECONDARY = {"combi_d4n15": secondary_combination, "batch": secondary_batch, "batch128": secondary_batch,
             "batch_d4n13": secondary_batch, "grad_d4n10": secondary_grad}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform of one grid, or of a combination set, "
              "runs on a single device here (sharding across GPUs is not built); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1309_0392_amd import sgh
    from paper_1309_0392_amd import workloads as W

    sgh.lib()  # fails loudly if the HIP library is not built
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.workload in GRIDS:
        out = run_grid(args, torch, np, sgh, W, args.workload)
    else:
        out = SECONDARY[args.workload](args, torch, np, sgh, W, args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
