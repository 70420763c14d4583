"""Several small strided axes in one pass (the box launch) against the
oracle, on the paper's 10-dimensional anisotropic shape (the first axis
refined, nine axes of 3 points) and on other mixes of small axes.  The box
applies the same per-point updates in the same axis order as the oracle, so
FP64 results are compared bitwise where the schedule holds only tile, box and
pole launches; a fused tile + walk launch rounds the inverse and the
transpose in its own order, and is held to the 1e-14 tolerance.  FP32 storage
within 2e-6."""
import numpy as np
import pytest

from gpu_util import OP_NAME, ORACLE, TOL, gpu_run, rel_err
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(2,) * 10, (3,) + (2,) * 9, (5,) + (2,) * 9, (8,) + (2,) * 9, (9, 3, 3, 3, 3), (4, 4, 3, 3, 2),
          (7, 2, 7, 2), (14, 2, 2), (6, 3, 3, 5, 2, 2)]


def _has_box(op, levels, dtype):
    s = sgh.schedule(op, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
    return any(l["kind"] == "box" for l in s["launches"])


@pytest.mark.parametrize("levels", SHAPES, ids=lambda l: "x".join(map(str, l)))
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_box_matches_oracle(levels, dtype, op):
    x = W.uniform(levels, [60, len(levels)], dtype)
    got = gpu_run(op, x, levels)
    ref = ORACLE[op](x.astype(np.float64), levels)
    _compare(op, levels, x, got, ref, dtype)


def _compare(op, levels, x, got, ref, dtype):
    kinds = [l["kind"] for l in sgh.schedule(op, levels, sgh.F64 if dtype == np.float64 else sgh.F32)["launches"]]
    if dtype == np.float64 and (op == sgh.OP_HIERARCHIZE or "tw" not in kinds):
        np.testing.assert_array_equal(got, ref)
    else:
        assert rel_err(op, x.astype(np.float64), got, ref) <= TOL[dtype]


def test_shapes_use_the_box():
    for levels in SHAPES[:5]:
        assert _has_box(sgh.OP_HIERARCHIZE, levels, np.float64), levels


@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_ten_dimensional_level12_f64(op):
    # 4095 x 3^9 = 80,601,885 points (645 MB FP64): a fused tile + walk launch
    # for axes 0-1, then boxes of axes 2-6 and 7-9
    levels = (12,) + (2,) * 9
    sched = sgh.schedule(op, levels)
    assert [l["kind"] for l in sched["launches"]].count("box") == 2 and sched["hbm_round_trips"] == 3
    x = W.uniform(levels, [61, 0])
    print("10-d level-12 grid, %s" % OP_NAME[op], flush=True)
    got = gpu_run(op, x, levels)
    _compare(op, levels, x, got, ORACLE[op](x, levels), np.float64)
