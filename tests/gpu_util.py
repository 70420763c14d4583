"""Helpers shared by the GPU tests (comparison against the CPU oracle)."""
import numpy as np
import torch

import oracle
from paper_1309_0392_amd import sgh

ORACLE = {sgh.OP_HIERARCHIZE: oracle.hierarchize,
          sgh.OP_DEHIERARCHIZE: oracle.dehierarchize,
          sgh.OP_ADJOINT: oracle.hierarchize_adjoint}
OP_NAME = {sgh.OP_HIERARCHIZE: "hierarchize", sgh.OP_DEHIERARCHIZE: "dehierarchize", sgh.OP_ADJOINT: "adjoint"}

# Tolerances: FP64 results within 1e-14, FP32-storage results within 2e-6 of the
# FP64 oracle run on the same (upcast) inputs.  The scale is max|x_in| for the
# hierarchization; the inverse and the transpose can amplify (nodal values sum
# up to l surpluses per axis, the transpose gathers up to 2(l-1) children), so
# their scale is max(max|x_in|, max|y_ref|).
TOL = {np.float64: 1e-14, np.float32: 2e-6}


def scale_of(op, x, ref):
    s = float(np.max(np.abs(x))) if x.size else 0.0
    if op != sgh.OP_HIERARCHIZE and ref.size:
        s = max(s, float(np.max(np.abs(ref))))
    return max(s, 1e-300)


def gpu_run(op, x: np.ndarray, levels, device="cuda"):
    t = torch.from_numpy(np.ascontiguousarray(x)).to(device)
    sgh.transform(op, t, levels)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_err(op, x, got, ref):
    return float(np.max(np.abs(got.astype(np.float64) - ref))) / scale_of(op, x, ref) if ref.size else 0.0
