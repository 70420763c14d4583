"""The workloads at full size on the GPU, checked against the oracle.

The full-size grids (about 1 GB each) are compared with the whole-grid oracle
on every element, for every operation and element type, plus the round trip
dehierarchize(hierarchize(x)) = x.  The combination-technique batch (589
grids) is checked grid by grid against the whole-grid oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, gpu_run, rel_err, scale_of
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu


def sample_positions(levels, count, seed):
    rng = np.random.default_rng(seed)
    pos = np.stack([rng.integers(1, 1 << l, size=count) for l in levels], axis=1)
    # always include the corners and the centre (boundary-adjacent predecessors, root)
    extra = [[1] * len(levels), [(1 << l) - 1 for l in levels], [1 << (l - 1) for l in levels]]
    return np.concatenate([pos, np.array(extra)], axis=0)


def test_small_2d_round_trip():
    levels = W.SMALL_2D
    x = W.uniform(levels, 0)
    h = gpu_run(sgh.OP_HIERARCHIZE, x, levels)
    assert rel_err(0, x, h, oracle.hierarchize(x, levels)) <= 1e-14
    back = gpu_run(sgh.OP_DEHIERARCHIZE, h, levels)
    assert np.max(np.abs(back - x)) <= 1e-14 * np.max(np.abs(x))


@pytest.mark.parametrize("name", ["aniso3d", "aniso5d"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_full_size_every_element(name, dtype):
    """The benchmark grids at full size, in the launch configuration bench.py
    times, against the whole-grid oracle on every element, for all three
    operations (a sampled pre-check of 300 points comes first, so that a gross
    error names itself quickly)."""
    if name == "aniso3d":
        levels, x = W.ANISO_3D, W.sine_plus_noise(W.ANISO_3D, seed=1)
    else:
        levels, x = W.ANISO_5D, W.uniform(W.ANISO_5D, seed=2)
    x = x.astype(dtype)
    x64 = x.astype(np.float64)
    xmax = float(np.max(np.abs(x64)))
    pos = sample_positions(levels, 300, seed=17)
    idx = tuple((pos[:, k] - 1) for k in reversed(range(len(levels))))
    dev = torch.from_numpy(x).cuda()
    print("full size %s %s: %d points" % (name, np.dtype(dtype).name, dev.numel()), flush=True)
    for op in (sgh.OP_HIERARCHIZE, sgh.OP_ADJOINT, sgh.OP_DEHIERARCHIZE):
        sched = [l["kind"] for l in sgh.schedule(op, levels, sgh.F64 if dtype == np.float64 else sgh.F32)["launches"]]
        t = dev.clone()
        sgh.transform(op, t, levels)
        torch.cuda.synchronize()
        got = t.cpu().numpy()
        del t
        pre = oracle.point(OP_NAME[op], x64, levels, pos)
        pre_err = float(np.max(np.abs(got[idx].astype(np.float64) - pre))) / scale_of(op, x64, pre)
        assert pre_err <= TOL[dtype], (OP_NAME[op], "sampled", pre_err)
        ref = ORACLE[op](x64, levels)
        err = rel_err(op, x64, got, ref)
        err_in = float(np.max(np.abs(got.astype(np.float64) - ref))) / xmax
        print("  %s %s: max error / scale %.3e, / max|x| %.3e" % (OP_NAME[op], "+".join(sched), err, err_in),
              flush=True)
        assert err <= TOL[dtype], (OP_NAME[op], err)
        del got, ref
    # round trip over every element
    t = dev.clone()
    sgh.hierarchize(t, levels)
    sgh.dehierarchize(t, levels)
    torch.cuda.synchronize()
    rt = float(torch.max(torch.abs(t - dev)).item()) / xmax
    print("  round trip err %.3e" % rt, flush=True)
    assert rt <= (1e-14 if dtype == np.float64 else 4e-6)


@pytest.mark.parametrize("name", ["aniso3d", "aniso5d"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_full_size_out_of_place(name, dtype):
    """The benchmark grids hierarchized out of place in the launch
    configuration `bench.py --out-of-place` times ((10,9,8): one fused launch
    with the axis after the walked one folded in), against the whole-grid
    oracle on every element; the source stays untouched."""
    if name == "aniso3d":
        levels, x = W.ANISO_3D, W.sine_plus_noise(W.ANISO_3D, seed=1)
    else:
        levels, x = W.ANISO_5D, W.uniform(W.ANISO_5D, seed=2)
    x = x.astype(dtype)
    x64 = x.astype(np.float64)
    sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, sgh.F64 if dtype == np.float64 else sgh.F32,
                         out_of_place=True)["launches"]
    if name == "aniso3d":
        assert len(sched) == 1 and sched[0]["outer_level"] == 8, sched
    src = torch.from_numpy(x).cuda()
    keep = src.clone()
    dst = torch.empty_like(src)
    sgh.transform_out(sgh.OP_HIERARCHIZE, src, dst, levels)
    torch.cuda.synchronize()
    assert torch.equal(src, keep)
    del keep
    got = dst.cpu().numpy()
    del dst, src
    ref = ORACLE[sgh.OP_HIERARCHIZE](x64, levels)
    err = rel_err(sgh.OP_HIERARCHIZE, x64, got, ref)
    print("full size out of place %s %s (%d launches): max error / max|x| %.3e"
          % (name, np.dtype(dtype).name, len(sched), err), flush=True)
    assert err <= TOL[dtype], err


def combi(dtype):
    lv, coef = W.combination_set()
    xs = W.combination_values(lv, seed=3, dtype=dtype)
    return lv, coef, xs


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("graph", [True, False], ids=["graph", "nograph"])
def test_combination_batch_plan(dtype, graph):
    lv, _, xs = combi(dtype)
    assert len(lv) == 589 and sum(x.size for x in xs) == 980797
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    ph = sgh.Plan(sgh.OP_HIERARCHIZE, ts, lv, graph=graph)
    pd = sgh.Plan(sgh.OP_DEHIERARCHIZE, ts, lv, graph=graph)
    pa = sgh.Plan(sgh.OP_ADJOINT, ts, lv, graph=graph)
    desc = ph.describe()
    assert desc["grids"] == 589 and desc["points"] == 980797 and desc["large"] == []
    # one batched launch holds the whole set: it is issued directly, not replayed from a graph
    assert len(desc["batches"]) == 1 and desc["graph"] is False
    refs = {op: [ORACLE[op](x.astype(np.float64), l) for x, l in zip(xs, lv)] for op in ORACLE}
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        for plan, op in ((ph, sgh.OP_HIERARCHIZE), (pd, sgh.OP_DEHIERARCHIZE), (pa, sgh.OP_ADJOINT)):
            for t, x in zip(ts, xs):
                t.copy_(torch.from_numpy(x))
            plan.execute()
            scratch.mul_(1.0001)  # unrelated eager work between replays
            torch.cuda.synchronize()
            worst = 0.0
            for t, x, r in zip(ts, xs, refs[op]):
                worst = max(worst, rel_err(op, x.astype(np.float64), t.cpu().numpy(), r))
            print("rep %d %s %s graph=%s worst err %.3e" % (rep, OP_NAME[op], dtype.__name__, graph, worst), flush=True)
            assert worst <= TOL[dtype]
    for p in (ph, pd, pa):
        p.close()


def test_batch_equals_per_grid_and_set_data():
    lv, _, xs = combi(np.float64)
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    per = [torch.from_numpy(x.copy()).cuda() for x in xs]
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, ts, lv, graph=True)
    plan.execute()
    for t, l in zip(per, lv):
        sgh.hierarchize(t, l)
    torch.cuda.synchronize()
    for a, b in zip(ts, per):
        assert torch.equal(a, b)
    # repoint to fresh buffers in shuffled memory order
    order = np.random.default_rng(0).permutation(len(lv))
    fresh = [None] * len(lv)
    for i in order:
        fresh[i] = torch.from_numpy(xs[i].copy()).cuda()
    plan.set_data(fresh)
    plan.execute()
    torch.cuda.synchronize()
    for a, b in zip(fresh, per):
        assert torch.equal(a, b)
    plan.close()


def test_plan_with_large_and_mixed_grids():
    lv = [(10, 9, 4), (3, 3), (2, 5, 1), (7, 7)]
    dts = [np.float64, np.float32, np.float64, np.float64]
    xs = [W.uniform(l, [40, i], d) for i, (l, d) in enumerate(zip(lv, dts))]
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    scratch = torch.randn(1 << 20, device="cuda")
    for op in ORACLE:
        plan = sgh.Plan(op, ts, lv, graph=True)
        d = plan.describe()
        assert len(d["large"]) == 2 and sum(b["tasks"] for b in d["batches"]) == 2
        assert d["graph"] is True  # several launches: replayed from one graph
        refs = [ORACLE[op](x.astype(np.float64), l) for x, l in zip(xs, lv)]
        for rep in range(3):
            for t, x in zip(ts, xs):
                t.copy_(torch.from_numpy(x))
            plan.execute()
            scratch.mul_(1.0001)  # unrelated eager work between replays
            torch.cuda.synchronize()
            for t, x, l, dt, ref in zip(ts, xs, lv, dts, refs):
                assert rel_err(op, x.astype(np.float64), t.cpu().numpy(), ref) <= TOL[dt], (OP_NAME[op], l, rep)
        plan.close()


def test_autotuned_plan_matches():
    lv, _, xs = combi(np.float32)
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, ts, lv, graph=True, autotune=True)
    plan.execute()
    torch.cuda.synchronize()
    for t, x, l in zip(ts, xs, lv):
        assert rel_err(0, x.astype(np.float64), t.cpu().numpy(), oracle.hierarchize(x.astype(np.float64), l)) <= 2e-6
    plan.close()


def test_flat_plan_equals_plan_and_rebases():
    """A relative plan gives the plan's results bit for bit, on two different
    buffers of the same layout (no re-upload between them)."""
    lv, _, xs = combi(np.float64)
    lv = lv + [(10, 9, 4), (7, 7)]  # plus grids beyond the tile (one-shot launches, rebased per call)
    xs = xs + [W.uniform(l, [41, i]) for i, l in enumerate(lv[-2:])]
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    for op in ORACLE:
        plan = sgh.Plan(op, ts, lv, graph=False)
        flat = sgh.FlatPlan(op, lv, sgh.F64)
        for t, x in zip(ts, xs):
            t.copy_(torch.from_numpy(x))
        plan.execute()
        for rep in range(2):
            buf = torch.empty(flat.total + 64 * rep, dtype=torch.float64, device="cuda")[64 * rep:]
            for v, x in zip(flat.views(buf), xs):
                v.copy_(torch.from_numpy(x))
            flat.execute(buf)
            torch.cuda.synchronize()
            for a, b in zip(flat.views(buf), ts):
                assert torch.equal(a, b), OP_NAME[op]
        # out of place: the source buffer is unchanged; the small grids equal the
        # plan bit for bit, the large ones (whose hierarchization may fold an axis
        # into the fused launch) the oracle within tolerance
        src = torch.empty(flat.total, dtype=torch.float64, device="cuda")
        for v, x in zip(flat.views(src), xs):
            v.copy_(torch.from_numpy(x))
        keep = src.clone()
        dst = torch.full_like(src, float("nan"))
        flat.execute_out(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, keep)
        for i, (a, b, x, l) in enumerate(zip(flat.views(dst), ts, xs, lv)):
            if i < len(lv) - 2:
                assert torch.equal(a, b), OP_NAME[op]
            else:
                assert rel_err(op, x, a.cpu().numpy(), ORACLE[op](x, l)) <= TOL[np.float64], (OP_NAME[op], l)
        # a relative plan refuses the plain execute
        assert sgh.lib().sgh_plan_execute(flat._h, None) == sgh.ERR_ARG
        plan.close()
        flat.close()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_size_classes_bitwise_equal_to_one_launch(dtype):
    """Size-classed batch launches apply the same per-point updates as one
    launch: results equal bit for bit, and equal the oracle within tolerance."""
    lv, _, xs = combi(dtype)
    ts1 = [torch.from_numpy(x.copy()).cuda() for x in xs]
    ts2 = [torch.from_numpy(x.copy()).cuda() for x in xs]
    try:
        for op in ORACLE:
            sgh.set_batch_classes(0, 1)
            p1 = sgh.Plan(op, ts1, lv, graph=False)
            sgh.set_batch_classes(1, 1)
            p2 = sgh.Plan(op, ts2, lv, graph=False)
            es = 8 if dtype == np.float64 else 4
            classes = {min(b for b in (8192, 16384, 32768, 65536) if W.num_points(l) * es <= b) for l in lv}
            assert len(p1.describe()["batches"]) == 1 and len(p2.describe()["batches"]) == len(classes) > 1
            for t1, t2, x in zip(ts1, ts2, xs):
                t1.copy_(torch.from_numpy(x))
                t2.copy_(torch.from_numpy(x))
            p1.execute()
            p2.execute()
            torch.cuda.synchronize()
            for t1, t2, x, l in zip(ts1, ts2, xs, lv):
                assert torch.equal(t1, t2), (OP_NAME[op], l)
            worst = max(rel_err(op, x.astype(np.float64), t.cpu().numpy(), ORACLE[op](x.astype(np.float64), l))
                        for t, x, l in zip(ts2, xs, lv))
            assert worst <= TOL[dtype]
            p1.close()
            p2.close()
    finally:
        sgh.set_batch_classes()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_size_classes_concurrent_graph_replays(dtype):
    """Size classes on forked streams, with a grid beyond the tile, captured in
    one graph: every replay (eager work on the stream between replays) equals
    the classes issued one after another on one stream, bit for bit."""
    lv, _, xs = combi(dtype)
    lv = lv + [(10, 9, 3)]
    xs = xs + [W.uniform((10, 9, 3), 61, dtype)]
    ta = [torch.from_numpy(x.copy()).cuda() for x in xs]
    tb = [torch.from_numpy(x.copy()).cuda() for x in xs]
    scratch = torch.randn(1 << 20, device="cuda")
    try:
        for op in ORACLE:
            sgh.set_batch_classes(1, 1, 0)
            serial = sgh.Plan(op, tb, lv, graph=False)
            sgh.set_batch_classes(1, 1, 1)
            forked = sgh.Plan(op, ta, lv, graph=True)
            d = forked.describe()
            assert len(d["batches"]) > 1 and d["graph"] is True
            for t, x in zip(tb, xs):
                t.copy_(torch.from_numpy(x))
            serial.execute()
            for rep in range(3):
                for t, x in zip(ta, xs):
                    t.copy_(torch.from_numpy(x))
                forked.execute()
                scratch.mul_(1.0001)
                torch.cuda.synchronize()
                for i, (a, b) in enumerate(zip(ta, tb)):
                    assert torch.equal(a, b), (OP_NAME[op], rep, lv[i])
            serial.close()
            forked.close()
    finally:
        sgh.set_batch_classes()
