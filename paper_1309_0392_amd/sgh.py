"""Thin Python binding of the C ABI in include/sgh.h (argument marshalling only).

Every transform runs in the HIP kernels of libsgh.so; there is no CPU or
PyTorch fallback.  If the shared library is missing, importing a function
raises immediately.

Tensors: a grid of level vector ``levels = (l_0, ..., l_{d-1})`` is a
contiguous torch tensor on a HIP device with shape
``(2**l_{d-1}-1, ..., 2**l_0-1)`` (grid axis 0 is the last, contiguous tensor
axis) and dtype float32 or float64.  Calls are asynchronous on the current
torch stream (or the stream given).
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import List, Optional, Sequence

MAX_DIM = 16
STATIC_TASKS = 4096  # grids per sgh_transform_batch_static call that fit the batch tile
MAX_LEVEL = 30
F32, F64 = 0, 1
OP_HIERARCHIZE, OP_DEHIERARCHIZE, OP_ADJOINT = 0, 1, 2
PLAN_GRAPH, PLAN_AUTOTUNE, PLAN_RELATIVE = 1, 2, 4

OK = 0
ERR_ARG, ERR_DTYPE, ERR_ALIGN, ERR_OVERLAP, ERR_HIP, ERR_NOMEM, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7

_PKG = os.path.dirname(os.path.abspath(__file__))
# SGH_LIBRARY may name another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("SGH_LIBRARY") or os.path.join(_PKG, "libsgh.so")


class SghGrid(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("level", ctypes.c_int32 * MAX_DIM),
        ("dtype", ctypes.c_int32),
        ("data", ctypes.c_void_p),
    ]


class SghError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed with %d (%s): %s" % (where, code, error_string(code) if _lib else "?", detail))
        self.code = code


_lib = None


def lib():
    """The loaded libsgh.so (ctypes.CDLL).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsgh.so not built: run `python -m paper_1309_0392_amd.build` "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        G = ctypes.POINTER(SghGrid)
        vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
        sig = {
            "sgh_hierarchize": ([G, i32, vp], ctypes.c_int),
            "sgh_dehierarchize": ([G, i32, vp], ctypes.c_int),
            "sgh_hierarchize_adjoint": ([G, i32, vp], ctypes.c_int),
            "sgh_transform": ([i32, G, i32, vp], ctypes.c_int),
            "sgh_transform_out": ([i32, G, G, i32, vp], ctypes.c_int),
            "sgh_transform_batch_static": ([i32, G, i32, vp], ctypes.c_int),
            "sgh_plan_execute_out": ([vp, vp, vp, vp], ctypes.c_int),
            "sgh_schedule_describe_out": ([i32, G, ctypes.c_char_p, i32], ctypes.c_int),
            "sgh_plan_create": ([ctypes.POINTER(vp), i32, G, i32, u32], ctypes.c_int),
            "sgh_plan_execute": ([vp, vp], ctypes.c_int),
            "sgh_plan_execute_at": ([vp, vp, vp], ctypes.c_int),
            "sgh_set_batch_classes": ([i32, i32, i32], ctypes.c_int),
            "sgh_set_outer_stencil": ([i32], ctypes.c_int),
            "sgh_set_xcd_order": ([i32], ctypes.c_int),
            "sgh_plan_set_data": ([vp, G, i32], ctypes.c_int),
            "sgh_plan_describe": ([vp, ctypes.c_char_p, i32], ctypes.c_int),
            "sgh_plan_destroy": ([vp], None),
            "sgh_validate": ([G, i32], ctypes.c_int),
            "sgh_num_points": ([G], i64),
            "sgh_schedule_describe": ([i32, G, ctypes.c_char_p, i32], ctypes.c_int),
            "sgh_error_string": ([ctypes.c_int], ctypes.c_char_p),
            "sgh_last_error_message": ([], ctypes.c_char_p),
            "sgh_version": ([], ctypes.c_char_p),
            "sgh_timing_enable": ([i32], ctypes.c_int),
            "sgh_set_pole_block": ([i32, i32], ctypes.c_int),
            "sgh_set_fusion": ([i32], ctypes.c_int),
            "sgh_set_pole_split": ([i32, i32, i32, i32], ctypes.c_int),
            "sgh_set_walk_preference": ([i32], ctypes.c_int),
            "sgh_set_split_spans": ([i32, i32], ctypes.c_int),
            "sgh_set_box_limits": ([i32, i32], ctypes.c_int),
            "sgh_set_medium_limits": ([i64, i32], ctypes.c_int),
            "sgh_timing_reset": ([], ctypes.c_int),
            "sgh_timing_report": ([ctypes.c_char_p, i32], ctypes.c_int),
            "sgh_combi_create": ([ctypes.POINTER(vp), G, i32, ctypes.POINTER(ctypes.c_double), u32],
                                 ctypes.c_int),
            "sgh_combi_sparse_points": ([vp], i64),
            "sgh_combi_num_subspaces": ([vp], i32),
            "sgh_combi_layout": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i64)], ctypes.c_int),
            "sgh_combi_gather": ([vp, vp, vp], ctypes.c_int),
            "sgh_combi_scatter": ([vp, vp, vp], ctypes.c_int),
            "sgh_combi_reduce": ([vp, vp, vp], ctypes.c_int),
            "sgh_combi_set_data": ([vp, G, i32], ctypes.c_int),
            "sgh_combi_destroy": ([vp], None),
            "sgh_sparse_layout": ([G, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                   ctypes.POINTER(i64)], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().sgh_error_string(int(code)).decode()


def last_error_message() -> str:
    return lib().sgh_last_error_message().decode()


def version() -> str:
    return lib().sgh_version().decode()


def _check(rc: int, where: str):
    if rc != OK:
        raise SghError(rc, where, last_error_message())


# --------------------------------------------------------------- descriptors
def make_grid(levels: Sequence[int], dtype: int, data_ptr: int) -> SghGrid:
    g = SghGrid()
    g.dim = len(levels)
    for k, l in enumerate(levels):
        g.level[k] = int(l)
    g.dtype = int(dtype)
    g.data = ctypes.c_void_p(int(data_ptr)) if data_ptr else None
    return g


def grid_array(grids: Sequence[SghGrid]):
    arr = (SghGrid * max(1, len(grids)))()
    for i, g in enumerate(grids):
        arr[i] = g
    return arr


def shape_of(levels: Sequence[int]):
    return tuple((1 << int(l)) - 1 for l in reversed(list(levels)))


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("grid tensors must be float32 or float64, got %s" % t.dtype)


def describe_tensor(t, levels) -> SghGrid:
    """Descriptor of a torch tensor holding the grid `levels` (validates shape/layout)."""
    if not t.is_cuda:
        raise ValueError("grid tensor must live on a HIP device")
    if tuple(t.shape) != shape_of(levels):
        raise ValueError("tensor shape %s does not match levels %s (expected %s)"
                         % (tuple(t.shape), tuple(levels), shape_of(levels)))
    if not t.is_contiguous():
        raise ValueError("grid tensor must be contiguous")
    return make_grid(levels, _dtype_code(t), t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _levels_list(tensors, levels):
    if levels and isinstance(levels[0], int):
        levels = [levels] * len(tensors)
    if len(levels) != len(tensors):
        raise ValueError("need one level vector per tensor")
    return levels


# ----------------------------------------------------------------- transforms
def transform(op: int, tensors, levels, stream=None):
    """Apply op in place to every tensor (one launch schedule per grid)."""
    if not isinstance(tensors, (list, tuple)):
        tensors = [tensors]
        levels = [levels]
    levels = _levels_list(tensors, levels)
    descs = [describe_tensor(t, l) for t, l in zip(tensors, levels)]
    _check(lib().sgh_transform(op, grid_array(descs), len(descs), _stream_handle(stream)), "sgh_transform")
    return tensors


def transform_out(op: int, src, dst, levels, stream=None):
    """dst[i] = op(src[i]) (src unchanged); dst[i] may be src[i] itself (in place)."""
    if not isinstance(src, (list, tuple)):
        src, dst, levels = [src], [dst], [levels]
    levels = _levels_list(src, levels)
    if len(dst) != len(src):
        raise ValueError("need one destination per source")
    sd = [describe_tensor(t, l) for t, l in zip(src, levels)]
    dd = [describe_tensor(t, l) for t, l in zip(dst, levels)]
    for a, b in zip(src, dst):
        if a.dtype != b.dtype:
            raise ValueError("source and destination dtypes differ")
    _check(lib().sgh_transform_out(op, grid_array(sd), grid_array(dd), len(sd), _stream_handle(stream)),
           "sgh_transform_out")
    return dst


def hierarchize(tensors, levels, stream=None):
    return transform(OP_HIERARCHIZE, tensors, levels, stream)


def dehierarchize(tensors, levels, stream=None):
    return transform(OP_DEHIERARCHIZE, tensors, levels, stream)


def hierarchize_adjoint(tensors, levels, stream=None):
    return transform(OP_ADJOINT, tensors, levels, stream)


# -------------------------------------------------------------------- plans
class Plan:
    """A batched plan (sgh_plan_*): one launch (one workgroup per grid) for all grids that
    fit on chip, captured with the launches of larger grids into a HIP graph."""

    def __init__(self, op: int, tensors, levels, graph: bool = True, autotune: bool = False):
        levels = _levels_list(tensors, levels)
        self.op = op
        self.levels = [tuple(int(x) for x in l) for l in levels]
        self.n = len(tensors)
        descs = [describe_tensor(t, l) for t, l in zip(tensors, self.levels)]
        self._arr = grid_array(descs)
        handle = ctypes.c_void_p()
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0)
        _check(lib().sgh_plan_create(ctypes.byref(handle), op, self._arr, self.n, flags), "sgh_plan_create")
        self._h = handle

    def set_data(self, tensors):
        descs = [describe_tensor(t, l) for t, l in zip(tensors, self.levels)]
        if len(descs) != self.n:
            raise ValueError("plan has %d grids, got %d" % (self.n, len(descs)))
        self._arr = grid_array(descs)
        _check(lib().sgh_plan_set_data(self._h, self._arr, self.n), "sgh_plan_set_data")

    def execute(self, stream=None):
        _check(lib().sgh_plan_execute(self._h, _stream_handle(stream)), "sgh_plan_execute")

    def describe(self) -> dict:
        need = lib().sgh_plan_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(max(need, 1))
        lib().sgh_plan_describe(self._h, buf, len(buf))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sgh_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FlatPlan:
    """A relative plan (SGH_PLAN_RELATIVE) over a set of grids stored back to
    back, in list order, in one flat tensor of `total` elements: grid i is the
    slice [starts[i], starts[i] + size_i).  The tensor is named at each
    execution, so one plan serves every buffer of that layout."""

    def __init__(self, op: int, levels_list, dtype: int, autotune: bool = False):
        self.op = op
        self.levels = [tuple(int(x) for x in l) for l in levels_list]
        self.n = len(self.levels)
        self.dtype = int(dtype)
        esize = 8 if self.dtype == F64 else 4
        self.sizes = [int(np_prod((1 << l) - 1 for l in lv)) for lv in self.levels]
        self.starts = []
        off = 0
        for sz in self.sizes:
            self.starts.append(off)
            off += sz
        self.total = off
        descs = [make_grid(lv, self.dtype, 0) for lv in self.levels]
        for g, st in zip(descs, self.starts):
            g.data = ctypes.c_void_p(st * esize) if st else None
        self._arr = grid_array(descs)
        handle = ctypes.c_void_p()
        flags = PLAN_RELATIVE | (PLAN_AUTOTUNE if autotune else 0)
        _check(lib().sgh_plan_create(ctypes.byref(handle), op, self._arr, self.n, flags), "sgh_plan_create")
        self._h = handle

    def views(self, flat):
        """The grids of a flat tensor, as views of their shapes."""
        return [flat[a:a + n].view(shape_of(lv)) for a, n, lv in zip(self.starts, self.sizes, self.levels)]

    def _check_flat(self, flat):
        import torch
        want = torch.float64 if self.dtype == F64 else torch.float32
        if flat.dtype != want or not flat.is_cuda or not flat.is_contiguous() or flat.numel() != self.total:
            raise ValueError("flat buffer must be a contiguous %s device tensor of %d elements" % (want, self.total))

    def execute(self, flat, stream=None):
        self._check_flat(flat)
        _check(lib().sgh_plan_execute_at(self._h, ctypes.c_void_p(flat.data_ptr()), _stream_handle(stream)),
               "sgh_plan_execute_at")
        return flat

    def execute_out(self, src, dst, stream=None):
        """dst = op(src) for every grid of the layout (src unchanged)."""
        self._check_flat(src)
        self._check_flat(dst)
        _check(lib().sgh_plan_execute_out(self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                          _stream_handle(stream)), "sgh_plan_execute_out")
        return dst

    def describe(self) -> dict:
        need = lib().sgh_plan_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(max(need, 1))
        lib().sgh_plan_describe(self._h, buf, len(buf))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sgh_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def np_prod(values) -> int:
    p = 1
    for v in values:
        p *= int(v)
    return p


# ------------------------------------------------------ combination technique
class Combination:
    """The sparse grid of a combination set (sgh_combi_*): gather of the grids'
    surpluses into the sparse grid, scatter back, and the whole reduce step
    (hierarchize, gather, scatter, dehierarchize)."""

    def __init__(self, tensors, levels, coefs, graph: bool = True, autotune: bool = False):
        import numpy as np
        levels = _levels_list(tensors, levels)
        self.levels = [tuple(int(x) for x in l) for l in levels]
        self.n = len(tensors)
        if len(coefs) != self.n:
            raise ValueError("need one coefficient per grid")
        self.dtype = tensors[0].dtype
        self._arr = grid_array([describe_tensor(t, l) for t, l in zip(tensors, self.levels)])
        self._coefs = (ctypes.c_double * self.n)(*[float(c) for c in coefs])
        handle = ctypes.c_void_p()
        flags = (PLAN_GRAPH if graph else 0) | (PLAN_AUTOTUNE if autotune else 0)
        _check(lib().sgh_combi_create(ctypes.byref(handle), self._arr, self.n, self._coefs, flags),
               "sgh_combi_create")
        self._h = handle
        self.sparse_points = int(lib().sgh_combi_sparse_points(self._h))
        nsub = int(lib().sgh_combi_num_subspaces(self._h))
        d = len(self.levels[0])
        sub = np.zeros((nsub, d), dtype=np.int32)
        off = np.zeros(nsub, dtype=np.int64)
        _check(lib().sgh_combi_layout(self._h, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "sgh_combi_layout")
        self.sub_levels, self.offsets = sub, off

    def new_sparse(self):
        """A device buffer for the sparse grid (uninitialized)."""
        import torch
        return torch.empty(self.sparse_points, dtype=self.dtype, device="cuda")

    def _sparse_ptr(self, sparse):
        if sparse.dtype != self.dtype or not sparse.is_cuda or not sparse.is_contiguous() \
                or sparse.numel() != self.sparse_points:
            raise ValueError("sparse buffer must be a contiguous %s device tensor of %d elements"
                             % (self.dtype, self.sparse_points))
        return ctypes.c_void_p(sparse.data_ptr())

    def gather(self, sparse, stream=None):
        _check(lib().sgh_combi_gather(self._h, self._sparse_ptr(sparse), _stream_handle(stream)),
               "sgh_combi_gather")
        return sparse

    def scatter(self, sparse, stream=None):
        _check(lib().sgh_combi_scatter(self._h, self._sparse_ptr(sparse), _stream_handle(stream)),
               "sgh_combi_scatter")

    def reduce(self, sparse, stream=None):
        _check(lib().sgh_combi_reduce(self._h, self._sparse_ptr(sparse), _stream_handle(stream)),
               "sgh_combi_reduce")
        return sparse

    def set_data(self, tensors):
        if len(tensors) != self.n:
            raise ValueError("set has %d grids, got %d" % (self.n, len(tensors)))
        self._arr = grid_array([describe_tensor(t, l) for t, l in zip(tensors, self.levels)])
        _check(lib().sgh_combi_set_data(self._h, self._arr, self.n), "sgh_combi_set_data")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().sgh_combi_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- host utils
def validate(grids: Sequence[SghGrid]) -> int:
    """sgh_validate on raw descriptors (host only); returns the code."""
    return lib().sgh_validate(grid_array(grids) if grids else None, len(grids))


def sparse_layout(levels_list, dtype: int = F64):
    """Host-side sparse-grid layout of a level set (sgh_sparse_layout):
    (subspace levels (S, d) int32, offsets (S,) int64, total points)."""
    import numpy as np
    descs = grid_array([make_grid(l, dtype, 0) for l in levels_list])
    n = len(levels_list)
    nsub, pts = ctypes.c_int32(), ctypes.c_int64()
    _check(lib().sgh_sparse_layout(descs, n, 0, None, None, ctypes.byref(nsub), ctypes.byref(pts)),
           "sgh_sparse_layout")
    d = len(levels_list[0])
    sub = np.zeros((nsub.value, d), dtype=np.int32)
    off = np.zeros(nsub.value, dtype=np.int64)
    _check(lib().sgh_sparse_layout(descs, n, nsub.value, sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(nsub),
                                   ctypes.byref(pts)), "sgh_sparse_layout")
    return sub, off, int(pts.value)


def num_points(levels, dtype: int = F64) -> int:
    g = make_grid(levels, dtype, 0)
    return int(lib().sgh_num_points(ctypes.byref(g)))


def schedule(op: int, levels, dtype: int = F64, out_of_place: bool = False) -> dict:
    """The launch schedule the library uses for one grid (host only), in place
    or out of place (transform_out)."""
    g = make_grid(levels, dtype, 0)
    fn = lib().sgh_schedule_describe_out if out_of_place else lib().sgh_schedule_describe
    need = fn(op, ctypes.byref(g), None, 0)
    if need < 0:
        _check(need, "sgh_schedule_describe")
    buf = ctypes.create_string_buffer(need)
    fn(op, ctypes.byref(g), buf, len(buf))
    return json.loads(buf.value.decode())


def set_pole_block(level: int, block_exponent: int):
    """Force the register block span 2**block_exponent for strided poles of `level` (0 = default)."""
    _check(lib().sgh_set_pole_block(int(level), int(block_exponent)), "sgh_set_pole_block")


def set_fusion(level: int):
    """1 (default): fuse the LDS-tile axes with one register-walked strided axis; 2: fused, two-level
    walk only; 0: one launch per pass."""
    _check(lib().sgh_set_fusion(int(level)), "sgh_set_fusion")


def set_split_spans(fine: int = 0, coarse: int = 0):
    """Block span exponents of the dyadic split of long poles (0 = default)."""
    _check(lib().sgh_set_split_spans(int(fine), int(coarse)), "sgh_set_split_spans")


def set_box_limits(max_bytes: int = 0, min_row_bytes: int = 0):
    """Size limits of the launches that transform runs of small strided axes together (0 = default)."""
    _check(lib().sgh_set_box_limits(int(max_bytes), int(min_row_bytes)), "sgh_set_box_limits")


def set_batch_classes(min_grids: int = 4096, min_per_class: int = 1024, concurrent: int = 0):
    """Plans: split the small grids of one dtype into size classes (one batch launch each) when there
    are at least min_grids of them (0 = never); classes below min_per_class grids join the next one;
    concurrent=1 overlaps the class launches on forked streams."""
    _check(lib().sgh_set_batch_classes(int(min_grids), int(min_per_class), int(concurrent)),
           "sgh_set_batch_classes")


def set_outer_stencil(on: int = 1):
    """Hierarchization: fold the axis after a fused three-level walk into that launch (1, default) or not (0)."""
    _check(lib().sgh_set_outer_stencil(int(on)), "sgh_set_outer_stencil")


def set_xcd_order(on: int = 0):
    """Fused launches: deal consecutive pencils to one XCD (1) or keep the hardware order (0, default)."""
    _check(lib().sgh_set_xcd_order(int(on)), "sgh_set_xcd_order")


def set_medium_limits(max_points: int = 1 << 18, min_grids: int = 16):
    """Plans: grids above the tile with at most max_points points go to the one-workgroup-per-grid
    launch when there are at least min_grids of them (max_points 0 turns it off)."""
    _check(lib().sgh_set_medium_limits(int(max_points), int(min_grids)), "sgh_set_medium_limits")


def set_walk_preference(pref: int):
    """0 (default): walk the qualifying strided axis with the smallest stride; 1: the largest."""
    _check(lib().sgh_set_walk_preference(int(pref)), "sgh_set_walk_preference")


def set_pole_split(level: int, top_exponent: int, block_exponent: int, prefetch: int = 0):
    """Force the three-level register walk for strided poles of `level` (block_exponent 0 = default)."""
    _check(lib().sgh_set_pole_split(int(level), int(top_exponent), int(block_exponent), int(prefetch)),
           "sgh_set_pole_split")


# (level, top exponent, block exponent) splits of the three-level pole walk and of the fused kernel
POLE3_SPLITS = [(7, 1, 3), (8, 2, 3), (9, 3, 3), (10, 2, 4)]
TW3_SPLITS = [(7, 1, 3), (8, 2, 3), (9, 3, 3)]


# POLE_PAIRS: (level, block exponent) pairs of the register-resident pole kernel
POLE_PAIRS = [(2, 2), (3, 3), (4, 4), (5, 5), (6, 6), (6, 3), (7, 4), (7, 3), (8, 4), (9, 5), (9, 4), (10, 5)]


# -------------------------------------------------------------------- timing
def timing_enable(on: bool = True):
    _check(lib().sgh_timing_enable(1 if on else 0), "sgh_timing_enable")


def timing_reset():
    _check(lib().sgh_timing_reset(), "sgh_timing_reset")


def timing_report() -> dict:
    need = lib().sgh_timing_report(None, 0)
    buf = ctypes.create_string_buffer(max(need, 2))
    lib().sgh_timing_report(buf, len(buf))
    return json.loads(buf.value.decode() or "{}")
