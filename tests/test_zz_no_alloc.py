"""The allocation-free batched entry point (sgh_transform_batch_static)
against the plan path it mirrors (sgh_plan_create + sgh_plan_execute without
autotuning): bit for bit, on two calls in a row, the second with a smaller
input, for every operation; and against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import OP_NAME, ORACLE, TOL, rel_err
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu


def static_call(op, ts, lv):
    arr = sgh.grid_array([sgh.describe_tensor(t, l) for t, l in zip(ts, lv)])
    return sgh.lib().sgh_transform_batch_static(op, arr, len(ts), sgh._stream_handle(None))


def cases():
    # first call: the d=4, n=10 set in FP64 plus a grid beyond the tile and an
    # FP32 grid; second call: a smaller, FP32 part of the set
    lv, _ = W.combination_set()
    big = lv + [(10, 9, 4), (5, 4)]
    big_x = W.combination_values(lv, seed=3) + [W.uniform((10, 9, 4), 51), W.uniform((5, 4), 52, np.float32)]
    small = lv[100:160]
    small_x = W.combination_values(small, seed=53, dtype=np.float32)
    return [(big, big_x), (small, small_x)]


@pytest.mark.parametrize("op", [sgh.OP_HIERARCHIZE, sgh.OP_DEHIERARCHIZE, sgh.OP_ADJOINT],
                         ids=["hierarchize", "dehierarchize", "adjoint"])
def test_static_equals_plan_on_two_calls(op):
    for call, (lv, xs) in enumerate(cases()):
        print("static call %d: %s, %d grids" % (call, OP_NAME[op], len(lv)), flush=True)
        a = [torch.from_numpy(x.copy()).cuda() for x in xs]
        b = [torch.from_numpy(x.copy()).cuda() for x in xs]
        assert static_call(op, a, lv) == sgh.OK, sgh.last_error_message()
        plan = sgh.Plan(op, b, lv, graph=False)
        plan.execute()
        torch.cuda.synchronize()
        for i, (ta, tb) in enumerate(zip(a, b)):
            assert torch.equal(ta, tb), (call, i, lv[i])
        plan.close()
        worst = max(rel_err(op, x.astype(np.float64), t.cpu().numpy(), ORACLE[op](x.astype(np.float64), l)) /
                    TOL[x.dtype.type] for x, t, l in zip(xs, a, lv))
        assert worst <= 1.0


def test_static_rejects_too_many_and_touches_nothing():
    n = sgh.STATIC_TASKS + 1
    ts = [torch.full((3,), float(i), dtype=torch.float64, device="cuda") for i in range(n)]
    before = [t.clone() for t in ts]
    assert static_call(0, ts, [(2,)] * n) == sgh.ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert all(torch.equal(t, u) for t, u in zip(ts, before))
