"""Poles too long for one on-chip pass (the dyadic block split) against the
oracle: contiguous poles beyond the LDS tile (level 14 and up, up to the 1 GiB
level-27 pole) and strided axes beyond the register kernels (level 11 and up).
Every point gets the same updates in the same order as in the oracle, so FP64
results are compared bitwise; FP32 storage within 2e-6 (hierarchization:
scale max|x|; inverse and transpose: max(max|x|, max|y_ref|))."""
import numpy as np
import pytest

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, gpu_run, rel_err
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(14,), (15,), (16,), (20,), (1, 14), (14, 3), (2, 12), (5, 12), (3, 13), (7, 11), (11, 11),
          (3, 2, 12), (13, 12)]


@pytest.mark.parametrize("levels", SHAPES, ids=lambda l: "x".join(map(str, l)))
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_split_matches_oracle(levels, dtype, op):
    sched = sgh.schedule(op, levels, sgh.F64 if dtype == np.float64 else sgh.F32)
    if dtype == np.float64 or max(levels) > 14:  # FP32 tiles hold a level-14 pole whole
        assert any(l["kind"] == "split" for l in sched["launches"]), sched
    x = W.uniform(levels, [50, len(levels)], dtype)
    got = gpu_run(op, x, levels)
    ref = ORACLE[op](x.astype(np.float64), levels)
    if dtype == np.float64:
        np.testing.assert_array_equal(got, ref)
    else:
        assert rel_err(op, x.astype(np.float64), got, ref) <= TOL[dtype]


@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_level27_pole_f64(op):
    # one pole of 2^27 - 1 points (1 GiB FP64): fine blocks of 2^13, then the
    # level-14 coarse pole (and, for the transpose, the root)
    levels = (27,)
    x = W.sine_plus_noise(levels, seed=6)
    print("level-27 pole, %s" % OP_NAME[op], flush=True)
    got = gpu_run(op, x, levels)
    ref = ORACLE[op](x, levels)
    np.testing.assert_array_equal(got, ref)


def test_level27_pole_f32():
    # every element against the whole-pole FP64 oracle on the upcast input, then the round trip
    levels = (27,)
    x = W.sine_plus_noise(levels, seed=7).astype(np.float32)
    x64 = x.astype(np.float64)
    for op in (sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT):
        print("level-27 FP32 pole, %s" % OP_NAME[op], flush=True)
        got = gpu_run(op, x, levels)
        err = rel_err(op, x64, got, ORACLE[op](x64, levels))
        print("  max error / scale %.3e" % err, flush=True)
        assert err <= TOL[np.float32]
    h = gpu_run(sgh.OP_HIERARCHIZE, x, levels)
    back = gpu_run(sgh.OP_DEHIERARCHIZE, h, levels)
    # FP32 round trip: a nodal value sums up to 27 surpluses
    assert np.max(np.abs(back.astype(np.float64) - x)) <= 27 * 2e-6 * np.abs(x).max()
