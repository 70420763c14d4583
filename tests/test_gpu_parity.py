"""GPU parity: every kernel path against the CPU oracle, element by element.

Shapes are chosen so that each launch schedule of the library runs: whole grid
in one LDS tile, LDS tile over the leading axes plus register-resident strided
poles (every supported block split), the dyadic split of long poles, runs of
small strided axes in one box launch, level-1 axes, and up to 16 dimensions."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, gpu_run, rel_err
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu

OPS = [sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT]
DTYPES = [np.float64, np.float32]

SHAPES = [
    # whole grid in one tile
    (1,), (2,), (5,), (13,), (5, 5), (3, 2, 4), (2, 2, 2, 2, 2, 2), (1, 3, 1, 2), (10, 3),
    # leading-axes tile + strided poles (FP64 tile capacity 8192 points)
    (7, 7), (10, 2), (10, 4, 3), (4, 4, 6), (3, 3, 3, 9), (5, 9), (2, 10, 2), (6, 8), (4, 10), (3, 5, 2, 5),
    # dyadic split: contiguous axis too long for a tile, strided axis too long for registers
    (14,), (3, 11), (2, 12, 2),
    # many dimensions, and the 10-d anisotropic stress shape (first axis grows, others 3 points)
    (2,) * 10, (6,) + (2,) * 9, (2, 2, 2, 2, 2, 2) + (1,) * 9 + (3,),
]


def ids(v):
    return "l" + "-".join(map(str, v))


@pytest.mark.parametrize("levels", SHAPES, ids=ids)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_parity_all_ops(levels, dtype):
    x = W.uniform(levels, [21, len(levels)], dtype)
    x64 = x.astype(np.float64)
    for op in OPS:
        ref = ORACLE[op](x64, levels)
        got = gpu_run(op, x, levels)
        err = rel_err(op, x64, got, ref)
        print("levels=%s dtype=%s op=%s err=%.3e" % (levels, dtype.__name__, OP_NAME[op], err), flush=True)
        assert err <= TOL[dtype], (OP_NAME[op], err)


@pytest.mark.parametrize("L,B", sgh.POLE_PAIRS)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_every_pole_block_split(L, B, dtype):
    """Every (level, block) variant of the register-resident strided kernel, at a
    stride large enough for full coalescing and at a tiny stride (ragged rows)."""
    sgh.set_pole_block(L, B)
    sgh.set_fusion(0)  # keep the strided axis in the pole kernel
    cap = 8192 if dtype == np.float64 else 16384  # points of the leading-axes LDS tile
    leads = [(12,) if dtype == np.float64 else (13,)]  # wide stride: 4095 / 8191 lanes per row
    if 31 * ((1 << L) - 1) > cap:
        leads.append((5,))  # stride 31: rows shorter than a wavefront
    try:
        for lead in leads:
            levels = lead + (L,)
            sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
            x = W.uniform(levels, [22, L, B], dtype)
            x64 = x.astype(np.float64)
            for op in OPS:
                ref = ORACLE[op](x64, levels)
                got = gpu_run(op, x, levels)
                err = rel_err(op, x64, got, ref)
                print("L=%d B=%d lead=%s op=%s err=%.3e sched=%s" % (L, B, lead, OP_NAME[op], err,
                      [l["kind"] for l in sched["launches"]]), flush=True)
                assert [l["kind"] for l in sched["launches"]] == ["tile", "pole"]
                assert sched["launches"][1]["B"] == B
                assert err <= TOL[dtype], (OP_NAME[op], err)
    finally:
        sgh.set_pole_block(L, 0)
        sgh.set_fusion(1)


def test_fp64_matches_oracle_bitwise_on_pole_and_tile_paths():
    """Same update order as the oracle, and 0.5*a is exact: FP64 results agree bit for bit
    when every axis has its own launch (the fused launch reorders axes, which only rounds
    differently)."""
    sgh.set_fusion(0)
    try:
        for levels in [(7, 7), (10, 4, 3), (5, 9), (3, 11), (4, 8), (2, 10, 2)]:
            x = W.uniform(levels, 5)
            for op in OPS:
                got = gpu_run(op, x, levels)
                assert np.array_equal(got, ORACLE[op](x, levels)), (levels, OP_NAME[op])
    finally:
        sgh.set_fusion(1)


def _tw_shape(ept, L, dtype):
    """A grid whose schedule fuses a leading tile of 1023 / 2047 / 4095 points with a
    walked strided axis of level L (the middle axis keeps the grid out of one tile;
    the tests prefer walking the largest stride, i.e. axis 2)."""
    lead = {1: 10, 2: 11, 4: 12}[ept]
    cap = 8192 if dtype == np.float64 else 16384
    mid = 2
    while ((1 << lead) - 1) * ((1 << mid) - 1) <= cap:
        mid += 1
    return (lead, mid, L)


TW_COMBOS = [(2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (7, 1), (8, 1), (9, 1), (2, 2), (3, 2), (4, 2), (5, 2),
             (6, 2), (2, 4), (3, 4), (4, 4), (5, 4)]


@pytest.mark.parametrize("fusion", [1, 2], ids=["default-walk", "two-level-walk"])
@pytest.mark.parametrize("L,ept", TW_COMBOS)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_fused_tile_walk(L, ept, dtype, fusion):
    """Fused tile + walked axis: every (walked level, tile elements per thread); the
    three-level walk (levels 7-9, one element per thread) and the two-level walk."""
    sgh.set_fusion(fusion)
    sgh.set_walk_preference(1)
    try:
        levels = _tw_shape(ept, L, dtype)
        sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
        tw = [l for l in sched["launches"] if l["kind"] == "tw" and l["axes"] == [0, 2]]
        three = fusion == 1 and ept == 1 and (L, L - 6, 3) in sgh.TW3_SPLITS
        two_level_built = L <= 8 and (ept == 1 or L <= 6)
        if not three and not two_level_built:
            assert not tw, sched  # no kernel walks this axis: it gets its own launch
            return
        assert len(tw) == 1 and tw[0]["axes"] == [0, 2] and tw[0]["ept"] == ept and tw[0]["L"] == L, sched
        assert tw[0]["split"] == (3 if three else 2), sched
        x = W.uniform(levels, [23, L, ept], dtype)
        x64 = x.astype(np.float64)
        for op in OPS:
            ref = ORACLE[op](x64, levels)
            got = gpu_run(op, x, levels)
            err = rel_err(op, x64, got, ref)
            print("tw levels=%s ept=%d split=%d op=%s err=%.3e" % (levels, ept, tw[0]["split"], OP_NAME[op], err),
                  flush=True)
            assert err <= TOL[dtype], (OP_NAME[op], err)
    finally:
        sgh.set_fusion(1)
        sgh.set_walk_preference(0)


@pytest.mark.parametrize("L,TB,B", sgh.POLE3_SPLITS)
@pytest.mark.parametrize("pf", [0, 1], ids=["nopf", "prefetch"])
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_every_pole3_split(L, TB, B, pf, dtype):
    """Three-level register walk of a strided pole, at a wide and (where the grid
    leaves the LDS tile) a 31-element stride."""
    sgh.set_pole_split(L, TB, B, pf)
    sgh.set_fusion(0)
    cap = 8192 if dtype == np.float64 else 16384
    leads = [(12,) if dtype == np.float64 else (13,)]
    if 31 * ((1 << L) - 1) > cap:
        leads.append((5,))
    try:
        for lead in leads:
            levels = lead + (L,)
            sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
            pole = sched["launches"][1]
            assert pole["kind"] == "pole" and pole["split"] == 3 and pole["TB"] == TB and pole["B"] == B
            assert pole["prefetch"] == pf
            x = W.uniform(levels, [25, L, pf], dtype)
            x64 = x.astype(np.float64)
            for op in OPS:
                ref = ORACLE[op](x64, levels)
                got = gpu_run(op, x, levels)
                err = rel_err(op, x64, got, ref)
                print("pole3 L=%d TB=%d B=%d pf=%d lead=%s op=%s err=%.3e" % (L, TB, B, pf, lead, OP_NAME[op], err),
                      flush=True)
                assert err <= TOL[dtype], (OP_NAME[op], err)
    finally:
        sgh.set_pole_split(L, 0, 0, 0)
        sgh.set_fusion(1)


@pytest.mark.parametrize("levels", [(6, 6, 3, 5), (3, 4, 5, 5), (10, 4, 9), (10, 4, 11), (10, 4, 3, 2),
                                    (5, 3, 2, 6, 2)], ids=ids)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_fused_tile_walk_layouts(levels, dtype):
    """Multi-axis tiles, a walked axis that is not the last one, and axes after it."""
    sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
    print(levels, [(l["kind"], l["axes"]) for l in sched["launches"]], flush=True)
    x = W.uniform(levels, [24, len(levels)], dtype)
    x64 = x.astype(np.float64)
    for op in OPS:
        ref = ORACLE[op](x64, levels)
        got = gpu_run(op, x, levels)
        assert rel_err(op, x64, got, ref) <= TOL[dtype], OP_NAME[op]


def test_deterministic_and_in_place_safe():
    levels = (9, 6, 5)
    x = W.uniform(levels, 3)
    a = gpu_run(sgh.OP_HIERARCHIZE, x, levels)
    b = gpu_run(sgh.OP_HIERARCHIZE, x, levels)
    assert np.array_equal(a, b)


def test_hat_function_exact_in_both_precisions():
    levels = (6, 5, 4)
    rng = np.random.default_rng(8)
    for dtype in DTYPES:
        for _ in range(4):
            m = [int(rng.integers(1, l + 1)) for l in levels]
            j = [int(2 * rng.integers(0, 1 << (mk - 1)) + 1) for mk in m]
            x = np.ones(W.shape_of(levels))
            for k, (l, mk, jk) in enumerate(zip(levels, m, j)):
                c = np.arange(1, 1 << l) / float(1 << l)
                v = np.maximum(0.0, 1.0 - np.abs(c * (1 << mk) - jk))
                view = [1] * len(levels)
                view[len(levels) - 1 - k] = v.size
                x = x * v.reshape(view)
            got = gpu_run(sgh.OP_HIERARCHIZE, x.astype(dtype), levels)
            expect = np.zeros_like(x)
            expect[tuple((jk << (l - mk)) - 1 for l, mk, jk in reversed(list(zip(levels, m, j))))] = 1.0
            assert np.array_equal(got.astype(np.float64), expect)


def test_many_grids_in_one_call_and_empty_call():
    lv = [(3, 4), (7, 7), (2, 2, 2), (5,)]
    xs = [W.uniform(l, [30, i]) for i, l in enumerate(lv)]
    ts = [torch.from_numpy(a.copy()).cuda() for a in xs]
    sgh.hierarchize(ts, lv)
    sgh.hierarchize([], [])
    torch.cuda.synchronize()
    for a, t, l in zip(xs, ts, lv):
        assert np.array_equal(t.cpu().numpy(), oracle.hierarchize(a, l))


def test_invalid_call_launches_nothing():
    """All-or-nothing validation: one bad descriptor -> error code, no grid touched."""
    good = torch.from_numpy(W.uniform((5, 5), 1)).cuda()
    before = good.clone()
    other = torch.zeros(100, dtype=torch.float64, device="cuda")
    descs = [sgh.describe_tensor(good, (5, 5)),
             sgh.make_grid((5, 5), sgh.F64, other.data_ptr() + 4)]        # misaligned
    rc = sgh.lib().sgh_hierarchize(sgh.grid_array(descs), 2, None)
    assert rc == sgh.ERR_ALIGN
    overlap = [sgh.describe_tensor(good, (5, 5)), sgh.make_grid((3,), sgh.F64, good.data_ptr() + 8)]
    assert sgh.lib().sgh_hierarchize(sgh.grid_array(overlap), 2, None) == sgh.ERR_OVERLAP
    torch.cuda.synchronize()
    assert torch.equal(good, before)
    # the library stays usable
    sgh.hierarchize(good, (5, 5))
    torch.cuda.synchronize()
    assert np.array_equal(good.cpu().numpy(), oracle.hierarchize(before.cpu().numpy(), (5, 5)))


def test_shape_checks_in_binding():
    t = torch.zeros((31, 31), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        sgh.hierarchize(t, (5, 4))
    with pytest.raises(ValueError):
        sgh.hierarchize(t.t(), (5, 5))
    with pytest.raises(TypeError):
        sgh.hierarchize(t.half(), (5, 5))


FOLDED = [(10, 7, 3), (10, 8, 2), (9, 9, 4), (10, 9, 1, 3), (10, 7, 5, 2), (8, 7, 6), (3, 3, 9, 5), (7, 8, 7)]


def gpu_run_out(op, x, levels):
    src = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    keep = src.clone()
    dst = torch.full_like(src, float("nan"))
    sgh.transform_out(op, src, dst, levels)
    torch.cuda.synchronize()
    assert torch.equal(src, keep)  # the source is left unchanged
    return dst.cpu().numpy()


@pytest.mark.parametrize("levels", FOLDED, ids=ids)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_folded_outer_axis(levels, dtype):
    """Out-of-place hierarchization with the axis after a three-level walk
    folded into the fused launch (its one-shot stencil applied as the rows are
    read): against the oracle, against the schedule with that axis in its own
    launch, and with the pencils dealt to XCDs in runs (the same arithmetic, bit
    for bit)."""
    code = sgh.F64 if dtype == np.float64 else sgh.F32
    sched = sgh.schedule(sgh.OP_HIERARCHIZE, levels, code, out_of_place=True)
    tw = sched["launches"][0]
    assert tw["kind"] == "tw" and tw["split"] == 3 and tw["outer_level"] > 0, sched
    x = W.uniform(levels, [29, len(levels)], dtype)
    x64 = x.astype(np.float64)
    ref = oracle.hierarchize(x64, levels)
    got = gpu_run_out(sgh.OP_HIERARCHIZE, x, levels)
    err = rel_err(sgh.OP_HIERARCHIZE, x64, got, ref)
    print("folded levels=%s %s: err %.3e" % (levels, np.dtype(dtype).name, err), flush=True)
    assert err <= TOL[dtype]
    try:
        sgh.set_xcd_order(1)
        assert sgh.schedule(sgh.OP_HIERARCHIZE, levels, code, out_of_place=True)["launches"][0]["xcd_order"] == 1
        np.testing.assert_array_equal(gpu_run_out(sgh.OP_HIERARCHIZE, x, levels), got)
        sgh.set_xcd_order(0)
        sgh.set_outer_stencil(0)
        assert sgh.schedule(sgh.OP_HIERARCHIZE, levels, code, out_of_place=True)["launches"][0]["outer_level"] == 0
        unfolded = gpu_run_out(sgh.OP_HIERARCHIZE, x, levels)
        assert float(np.max(np.abs(unfolded.astype(np.float64) - got))) <= 2 * TOL[dtype] * np.abs(x64).max()
    finally:
        sgh.set_xcd_order(0)
        sgh.set_outer_stencil(1)


OUT_SHAPES = [(5, 5), (10, 9, 3), (6, 6, 5, 5), (14,), (5, 12), (6,) + (2,) * 9, (10, 4, 3), (3, 2, 4)]


@pytest.mark.parametrize("levels", OUT_SHAPES, ids=ids)
@pytest.mark.parametrize("dtype", DTYPES, ids=["f64", "f32"])
def test_transform_out_all_ops(levels, dtype):
    """Out of place, every operation and schedule kind (tile, fused, pole,
    split, box): the destination equals the oracle and the source is unchanged;
    dst == src is the in-place transform."""
    x = W.uniform(levels, [31, len(levels)], dtype)
    x64 = x.astype(np.float64)
    for op in OPS:
        ref = ORACLE[op](x64, levels)
        got = gpu_run_out(op, x, levels)
        err = rel_err(op, x64, got, ref)
        print("out levels=%s %s %s: err %.3e" % (levels, np.dtype(dtype).name, OP_NAME[op], err), flush=True)
        assert err <= TOL[dtype], (OP_NAME[op], err)
        t = torch.from_numpy(x.copy()).cuda()
        sgh.transform_out(op, t, t, levels)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(t.cpu().numpy(), gpu_run(op, x, levels))
