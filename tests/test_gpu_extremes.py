"""The largest cases the library accepts, against the oracle: the top level
(30, a 4 GiB FP32 pole), a 2 GiB FP64 pole, and the maximum dimension (16 axes
of 3 points, 43 M points).  FP64 results are compared bitwise (the split and
tile paths keep the oracle's per-point order); the FP32 level-30 pole on every
element against the FP64 oracle on the upcast input, and by its round trip."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, gpu_run
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_top_level_pole_f32():
    # the level-30 FP32 pole (4 GiB) against the whole-pole FP64 oracle on every element
    levels = (sgh.MAX_LEVEL,)
    N = (1 << 30) - 1
    gen = torch.Generator(device="cuda")
    gen.manual_seed(70)
    x = torch.rand(N, dtype=torch.float32, device="cuda", generator=gen) * 2 - 1
    x0 = x.clone()
    print("level-30 FP32 pole (4 GiB)", flush=True)
    sgh.hierarchize(x, levels)
    torch.cuda.synchronize()
    xin = x0.cpu().numpy().astype(np.float64)
    xmax = float(np.abs(xin).max())
    ref = oracle.hierarchize(xin, levels)
    got = x.cpu().numpy()
    err = 0.0
    for a in range(0, N, 1 << 27):  # in slices, to bound the temporaries
        err = max(err, float(np.max(np.abs(got[a:a + (1 << 27)].astype(np.float64) - ref[a:a + (1 << 27)]))))
    del ref, got
    print("  max error / max|x| %.3e" % (err / xmax), flush=True)
    assert err <= TOL[np.float32] * xmax
    sgh.dehierarchize(x, levels)
    torch.cuda.synchronize()
    # a nodal value sums at most 30 surpluses, each within the FP32 rounding of the forward pass
    assert torch.max(torch.abs(x - x0)).item() <= 30 * TOL[np.float32]


@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_level28_pole_f64(op):
    levels = (28,)
    x = W.uniform(levels, 72)
    print("level-28 FP64 pole (2 GiB), %s" % OP_NAME[op], flush=True)
    np.testing.assert_array_equal(gpu_run(op, x, levels), ORACLE[op](x, levels))


@pytest.mark.parametrize("op", list(ORACLE), ids=[OP_NAME[o] for o in ORACLE])
def test_sixteen_dimensions_f64(op):
    levels = (2,) * sgh.MAX_DIM
    assert len(levels) == 16
    x = W.uniform(levels, 73)
    print("16-d grid of 3^16 points, %s" % OP_NAME[op], flush=True)
    got = gpu_run(op, x, levels)
    kinds = [l["kind"] for l in sgh.schedule(op, levels)["launches"]]
    ref = ORACLE[op](x, levels)
    if op == sgh.OP_HIERARCHIZE or "tw" not in kinds:
        np.testing.assert_array_equal(got, ref)
    else:
        assert np.max(np.abs(got - ref)) <= TOL[np.float64] * max(np.abs(x).max(), np.abs(ref).max())
