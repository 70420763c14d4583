"""CPU oracle for the hierarchization of combination grids (test infrastructure).

TEST INFRASTRUCTURE ONLY: only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double precision), which
follows Algorithm 1 of P. Hupp, "Hierarchization for the Sparse Grid
Combination Technique" (arXiv:1309.0392), Section 3.  This module only
marshals numpy arrays into it.

Array convention: a grid of level vector ``(l_0, ..., l_{d-1})`` is a
C-contiguous float64 array of shape ``(2**l_{d-1}-1, ..., 2**l_0-1)``; the last
numpy axis is grid axis 0, the fastest-changing index (the paper's x_1).

Parity status: every routine exported here is pinned: the transforms by
``tests/test_oracle_pins.py`` (hat basis, linear reproduction, dense hat-evaluation
matrices, sine closed form, axis-order invariance, dense transpose, brute-force flop
counts), the combination-technique gather / scatter by ``tests/test_oracle_combi.py``
(coefficient identity, surpluses of one function, unit surpluses, and the round trip
against the nodal combination formula sum_l c_l u_l).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP: the pole loops shared over the host's
# cores (used only to time the oracle on all cores; same arithmetic per pole)
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None
_lib_omp = None


def _compile(out: str, extra) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared"] + list(extra) + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, no fast-math) into liboracle.so, and the
    OpenMP build liboracle_omp.so."""
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, extra)
    return _LIB_PATH


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_int64)
    for name in ("oracle_hierarchize", "oracle_dehierarchize", "oracle_hierarchize_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [dp, ctypes.c_int, ip]
        f.restype = ctypes.c_int
    for name in ("oracle_hierarchize_axis", "oracle_dehierarchize_axis",
                 "oracle_hierarchize_adjoint_axis"):
        f = getattr(lib, name)
        f.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int]
        f.restype = ctypes.c_int
    for name in ("oracle_hierarchize_point", "oracle_dehierarchize_point",
                 "oracle_hierarchize_adjoint_point"):
        f = getattr(lib, name)
        f.argtypes = [dp, ctypes.c_int, ip, lp]
        f.restype = ctypes.c_double
    for name in ("oracle_flops_eq1", "oracle_mults_reduced"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, ip]
        f.restype = ctypes.c_double
    lib.oracle_num_points.argtypes = [ctypes.c_int, ip]
    lib.oracle_num_points.restype = ctypes.c_int64
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    return lib


def _load(threads: bool = False):
    global _lib, _lib_omp
    if threads:
        if _lib_omp is None:
            build()
            _lib_omp = _bind(ctypes.CDLL(_OMP_PATH))
        return _lib_omp
    if _lib is None:
        build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def num_threads(threads: bool = False) -> int:
    """Threads the pole loops use (1 for the plain build)."""
    return int(_load(threads).oracle_threads())


def shape_of(levels) -> tuple:
    """numpy shape of a grid: reversed (2**l - 1), axis 0 last."""
    return tuple((1 << int(l)) - 1 for l in reversed(list(levels)))


def _levels_arg(levels):
    lv = [int(l) for l in levels]
    return (ctypes.c_int * len(lv))(*lv), len(lv)


def _check(x: np.ndarray, levels):
    if x.dtype != np.float64 or not x.flags["C_CONTIGUOUS"]:
        raise TypeError("oracle works on C-contiguous float64 arrays")
    if tuple(x.shape) != shape_of(levels):
        raise ValueError("shape %s does not match levels %s" % (x.shape, tuple(levels)))


def _run(name, x, levels, *extra, threads: bool = False):
    lib = _load(threads)
    y = np.array(x, dtype=np.float64, order="C", copy=True)
    _check(y, levels)
    lv, d = _levels_arg(levels)
    rc = getattr(lib, name)(y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d, lv, *extra)
    if rc != 0:
        raise ValueError("%s rejected levels %s" % (name, tuple(levels)))
    return y


def hierarchize(x, levels, threads: bool = False) -> np.ndarray:
    """Algorithm 1 on a copy of x (float64); threads=True runs the poles of
    each direction on all cores (OpenMP build)."""
    return _run("oracle_hierarchize", x, levels, threads=threads)


def dehierarchize(x, levels, threads: bool = False) -> np.ndarray:
    return _run("oracle_dehierarchize", x, levels, threads=threads)


def hierarchize_adjoint(x, levels, threads: bool = False) -> np.ndarray:
    return _run("oracle_hierarchize_adjoint", x, levels, threads=threads)


def hierarchize_inplace(x: np.ndarray, levels, threads: bool = False) -> np.ndarray:
    """Algorithm 1 applied to x itself (C-contiguous float64), for timing the
    oracle without the copy the other entry points make."""
    _check(x, levels)
    lv, d = _levels_arg(levels)
    if _load(threads).oracle_hierarchize(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d, lv) != 0:
        raise ValueError("oracle_hierarchize rejected levels %s" % (tuple(levels),))
    return x


def hierarchize_adjoint_inplace(x: np.ndarray, levels, threads: bool = False) -> np.ndarray:
    _check(x, levels)
    lv, d = _levels_arg(levels)
    if _load(threads).oracle_hierarchize_adjoint(x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d, lv) != 0:
        raise ValueError("oracle_hierarchize_adjoint rejected levels %s" % (tuple(levels),))
    return x


def hierarchize_axis(x, levels, axis: int) -> np.ndarray:
    return _run("oracle_hierarchize_axis", x, levels, int(axis))


def dehierarchize_axis(x, levels, axis: int) -> np.ndarray:
    return _run("oracle_dehierarchize_axis", x, levels, int(axis))


def hierarchize_adjoint_axis(x, levels, axis: int) -> np.ndarray:
    return _run("oracle_hierarchize_adjoint_axis", x, levels, int(axis))


_POINT_FN = {
    "hierarchize": "oracle_hierarchize_point",
    "dehierarchize": "oracle_dehierarchize_point",
    "adjoint": "oracle_hierarchize_adjoint_point",
}


def point(op: str, x: np.ndarray, levels, positions) -> np.ndarray:
    """Outputs of ``op`` at the given points, each computed on its own.

    ``positions`` is an integer array of shape (P, d) of 1-based positions
    along grid axes 0..d-1.  x is read in place (no copy)."""
    lib = _load()
    if x.dtype != np.float64 or not x.flags["C_CONTIGUOUS"]:
        raise TypeError("oracle works on C-contiguous float64 arrays")
    if tuple(x.shape) != shape_of(levels):
        raise ValueError("shape does not match levels")
    fn = getattr(lib, _POINT_FN[op])
    lv, d = _levels_arg(levels)
    pos = np.ascontiguousarray(positions, dtype=np.int64).reshape(-1, d)
    xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = np.empty(pos.shape[0], dtype=np.float64)
    for r in range(pos.shape[0]):
        out[r] = fn(xp, d, lv, pos[r].ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def flops_eq1(levels) -> float:
    """Corrected Eq. (1) flop count of Algorithm 1."""
    lv, d = _levels_arg(levels)
    return _load().oracle_flops_eq1(d, lv)


def mults_reduced(levels) -> float:
    """Multiplications of the reduced-operation variant, M(d, l)."""
    lv, d = _levels_arg(levels)
    return _load().oracle_mults_reduced(d, lv)


def num_points(levels) -> int:
    lv, d = _levels_arg(levels)
    return int(_load().oracle_num_points(d, lv))


# ------------------------------------------------- combination technique ---
def sparse_layout(levels_list):
    """Sparse-grid storage of a combination set: every hierarchical subspace m
    (m >= 1) contained in at least one grid, ordered by |m|_1, then
    lexicographically (m_0 first); subspace m holds prod 2^(m_k - 1) points,
    axis 0 fastest.  Returns (subspace levels (S, d) int array, offsets (S,),
    total points)."""
    d = len(levels_list[0])
    subs = set()
    for lv in levels_list:
        ranges = [range(1, int(l) + 1) for l in lv]
        stack = [()]
        for r in ranges:
            stack = [t + (v,) for t in stack for v in r]
        subs.update(stack)
    order = sorted(subs, key=lambda m: (sum(m), m))
    sub_levels = np.array(order, dtype=np.int32).reshape(-1, d)
    sizes = np.array([1 << (sum(m) - d) for m in order], dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    return sub_levels, offsets, int(sizes.sum())


def _combi_args(xs, levels_list):
    lib = _load()
    d = len(levels_list[0])
    arrays = [np.ascontiguousarray(x, dtype=np.float64) for x in xs]
    for a, lv in zip(arrays, levels_list):
        if tuple(a.shape) != shape_of(lv):
            raise ValueError("grid shape does not match its levels")
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(arrays))(
        *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrays])
    lv = np.ascontiguousarray(np.array(levels_list, dtype=np.int32).reshape(-1))
    return lib, d, arrays, ptrs, lv


def combi_gather(xs, levels_list, coefs, layout=None) -> np.ndarray:
    """Sparse-grid surpluses: sum over grids (in list order) of coef * grid surplus."""
    lib, d, arrays, ptrs, lv = _combi_args(xs, levels_list)
    sub, off, total = layout if layout is not None else sparse_layout(levels_list)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.int64)
    c = np.ascontiguousarray(coefs, dtype=np.float64)
    out = np.zeros(total, dtype=np.float64)
    f = lib.oracle_combi_gather
    f.restype = ctypes.c_int
    rc = f(len(arrays), ptrs, lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
           c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), d, sub.shape[0],
           sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
           ctypes.c_int64(total), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_combi_gather failed (%d)" % rc)
    return out


def combi_scatter(sparse, levels_list, layout=None):
    """Grids whose every point holds the sparse grid's surplus at that point."""
    xs = [np.zeros(shape_of(lv)) for lv in levels_list]
    lib, d, arrays, ptrs, lv = _combi_args(xs, levels_list)
    sub, off, total = layout if layout is not None else sparse_layout(levels_list)
    sub = np.ascontiguousarray(sub, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.int64)
    sp = np.ascontiguousarray(sparse, dtype=np.float64)
    if sp.size != total:
        raise ValueError("sparse array has %d points, layout %d" % (sp.size, total))
    f = lib.oracle_combi_scatter
    f.restype = ctypes.c_int
    rc = f(len(arrays), ptrs, lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), d, sub.shape[0],
           sub.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
           sp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_combi_scatter failed (%d)" % rc)
    return arrays


def combi_round_trip(xs, levels_list, coefs):
    """Iterated combination technique step without a solver: hierarchize every
    grid, gather the sparse grid, scatter it back, dehierarchize every grid."""
    hs = [hierarchize(x, lv) for x, lv in zip(xs, levels_list)]
    layout = sparse_layout(levels_list)
    sp = combi_gather(hs, levels_list, coefs, layout)
    back = combi_scatter(sp, levels_list, layout)
    return [dehierarchize(b, lv) for b, lv in zip(back, levels_list)], sp
