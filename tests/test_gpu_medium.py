"""Plans over many grids too large for one LDS tile: the medium launch (one
workgroup per grid, the grid's axes in passes through its tile) against the
oracle, grid by grid.

The medium kernel applies the same per-axis steps in the same axis order as
the oracle (Algorithm 1 along each axis; the inverse and the transpose in the
reverse axis order), so FP64 hierarchization is compared bit for bit; the
other cases are held to the tolerances of the other GPU parity tests."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, rel_err
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def default_limits():
    sgh.set_medium_limits()
    yield
    sgh.set_medium_limits()


def run_plan(op, xs, lv, graph, reps=1):
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    plan = sgh.Plan(op, ts, lv, graph=graph)
    desc = plan.describe()
    scratch = torch.randn(1 << 20, device="cuda")
    outs = []
    for _ in range(reps):
        for t, x in zip(ts, xs):
            t.copy_(torch.from_numpy(x))
        plan.execute()
        scratch.mul_(1.0001)  # unrelated eager work between replays
        torch.cuda.synchronize()
        outs.append([t.cpu().numpy() for t in ts])
    plan.close()
    return desc, outs


@pytest.mark.parametrize("op", list(ORACLE), ids=lambda o: OP_NAME[o])
def test_d4n11_set_f64(op):
    lv, _ = W.combination_set(4, 11)
    xs = W.combination_values(lv, seed=21)
    desc, outs = run_plan(op, xs, lv, graph=True, reps=2)
    med = sum(m["tasks"] for m in desc["medium"])
    print("d4n11 %s: %d grids, %d medium, %d large" % (OP_NAME[op], len(lv), med, len(desc["large"])), flush=True)
    assert med == 68 and desc["large"] == [] and desc["graph"] is True
    refs = [ORACLE[op](x, l) for x, l in zip(xs, lv)]
    for rep, got in enumerate(outs):
        worst, differ = 0.0, 0
        for x, ref, g in zip(xs, refs, got):
            worst = max(worst, rel_err(op, x, g, ref))
            differ += int(not np.array_equal(g, ref))
        print("  rep %d worst err %.3e, %d grids not bitwise" % (rep, worst, differ), flush=True)
        assert worst <= TOL[np.float64]
        if op == sgh.OP_HIERARCHIZE:
            assert differ == 0


@pytest.mark.parametrize("op", list(ORACLE), ids=lambda o: OP_NAME[o])
def test_d3n13_set_f32(op):
    lv, _ = W.combination_set(3, 13)
    xs = W.combination_values(lv, seed=22, dtype=np.float32)
    desc, outs = run_plan(op, xs, lv, graph=False)
    med = sum(m["tasks"] for m in desc["medium"])
    print("d3n13 f32 %s: %d grids, %d medium" % (OP_NAME[op], len(lv), med), flush=True)
    assert med == 55
    worst = 0.0
    for x, l, g in zip(xs, lv, outs[0]):
        x64 = x.astype(np.float64)
        worst = max(worst, rel_err(op, x64, g, ORACLE[op](x64, l)))
    print("  worst err %.3e" % worst, flush=True)
    assert worst <= TOL[np.float32]


# Shapes at the kernel's limits: an axis of 8191 points after a 3-point tile
# (one column per box), a full tile row followed by a short axis with ragged
# boxes, level-1 axes in between and two box passes, five axes, FP32 rows of
# 16383 points, two and three trailing axes sharing one box pass.
EDGE = [((2, 13), np.float64), ((13, 2), np.float64), ((3, 1, 11, 1, 2), np.float64),
        ((4, 3, 3, 3, 3), np.float64), ((12, 3), np.float64), ((14, 2), np.float32),
        ((2, 14), np.float32), ((5, 5, 5), np.float32), ((1, 9, 6), np.float64),
        ((6, 6, 2, 2), np.float64), ((7, 2, 2, 2, 2, 2, 2), np.float32), ((9, 3, 2, 2, 2), np.float64)]


@pytest.mark.parametrize("op", list(ORACLE), ids=lambda o: OP_NAME[o])
def test_edge_shapes_forced(op):
    sgh.set_medium_limits(1 << 18, 1)
    lv = [l for l, _ in EDGE]
    xs = [W.uniform(l, [23, i], dt) for i, (l, dt) in enumerate(EDGE)]
    desc, outs = run_plan(op, xs, lv, graph=True, reps=2)
    med = sum(m["tasks"] for m in desc["medium"])
    assert med == len(EDGE) and desc["large"] == [] and desc["batches"] == []
    for rep, got in enumerate(outs):
        for x, (l, dt), g in zip(xs, EDGE, got):
            x64 = x.astype(np.float64)
            ref = ORACLE[op](x64, l)
            err = rel_err(op, x64, g, ref)
            if dt == np.float64 and op == sgh.OP_HIERARCHIZE:
                assert np.array_equal(g, ref), (l, rep)
            assert err <= TOL[dt], (OP_NAME[op], l, rep, err)


def test_medium_equals_per_grid_launches():
    lv, _ = W.combination_set(4, 11)
    xs = W.combination_values(lv, seed=24)
    for op in ORACLE:
        sgh.set_medium_limits()
        d1, (a,) = run_plan(op, xs, lv, graph=False)
        sgh.set_medium_limits(0, 16)  # off: every medium grid gets its own launches
        d2, (b,) = run_plan(op, xs, lv, graph=False)
        assert d1["medium"] and not d2["medium"] and len(d2["large"]) == d1["medium"][0]["tasks"]
        worst = max(rel_err(op, x, u, v) for x, u, v in zip(xs, a, b))
        print("%s medium vs per-grid launches: %.3e" % (OP_NAME[op], worst), flush=True)
        assert worst <= 2 * TOL[np.float64]


def test_below_min_count_goes_large_and_set_data():
    lv = [(7, 7), (9, 6), (3, 12)]
    xs = [W.uniform(l, [25, i]) for i, l in enumerate(lv)]
    ts = [torch.from_numpy(x.copy()).cuda() for x in xs]
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, ts, lv, graph=True)
    assert plan.describe()["medium"] == [] and len(plan.describe()["large"]) == 3
    plan.close()
    sgh.set_medium_limits(1 << 18, 3)
    plan = sgh.Plan(sgh.OP_HIERARCHIZE, ts, lv, graph=True)
    assert plan.describe()["medium"][0]["tasks"] == 3
    fresh = [torch.from_numpy(x.copy()).cuda() for x in xs]
    plan.set_data(fresh)
    plan.execute()
    torch.cuda.synchronize()
    for t, f, x, l in zip(ts, fresh, xs, lv):
        assert np.array_equal(f.cpu().numpy(), oracle.hierarchize(x, l))
        assert np.array_equal(t.cpu().numpy(), x)  # the old buffers are untouched
    plan.close()
