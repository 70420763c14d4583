"""Combination technique on the GPU against the oracle: gather of surpluses
into the sparse grid, scatter back into the grids, and the reduce step
(hierarchize, gather, scatter, dehierarchize) with and without graph capture.

Gather sums the grids' coefficient-weighted values in list order with products
and sums rounded separately, as the oracle does, so FP64 gather is compared
bitwise; scatter only copies, so it is bitwise in both dtypes.  The reduce step
goes through the hierarchization kernels and is compared point by point within
bounds built from each point's own contributors (tests/combi_bounds.py): the
transform tolerances (FP64 1e-14, FP32 storage 2e-6 of the FP64 oracle on the
upcast inputs) weighted by the point's |coefficients|, the rounding of its
weighted sum, and, for grid points, the propagation through the inverse."""
import numpy as np
import pytest
import torch

import oracle
from combi_bounds import reduce_bounds, reduce_violations
from paper_1309_0392_amd import sgh
from paper_1309_0392_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-14, np.float32: 2e-6}
SETS = {
    "d2n5": lambda: W.combination_set(2, 5),
    "d3n6": lambda: W.combination_set(3, 6),
    "d4n10": lambda: W.combination_set(4, 10),
    "d5n7": lambda: W.combination_set(5, 7),
    "single": lambda: ([(4, 3, 2)], [1.0]),
    "d1": lambda: ([(9,)], [1.0]),
    "aniso_random_coefs": lambda: ([(6, 2), (5, 3), (3, 4), (2, 6), (1, 8), (4, 4)],
                                   [0.75, -1.5, 2.0, 0.3, -0.9, 1.25]),
}


def _to_dev(xs):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]


def _host(ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("name", list(SETS))
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_gather_matches_oracle(name, dtype):
    levels, coefs = SETS[name]()
    xs = W.combination_values(levels, seed=11, dtype=dtype)
    ts = _to_dev(xs)
    c = sgh.Combination(ts, levels, coefs, graph=False)
    osub, ooff, ototal = oracle.sparse_layout(levels)
    assert c.sparse_points == ototal
    np.testing.assert_array_equal(c.sub_levels, osub)
    np.testing.assert_array_equal(c.offsets, ooff)
    sp = c.new_sparse().fill_(float("nan"))
    c.gather(sp)
    got = sp.cpu().numpy()
    ref = oracle.combi_gather([x.astype(np.float64) for x in xs], levels, coefs)
    if dtype == np.float64:
        np.testing.assert_array_equal(got, ref)
    else:
        scale = max(float(max(np.abs(x).max() for x in xs)), 1e-300) * sum(abs(v) for v in coefs)
        assert np.isfinite(got).all()
        assert np.max(np.abs(got - ref)) <= TOL[dtype] * scale
    # the grids are untouched by a gather
    for x, t in zip(xs, _host(ts)):
        np.testing.assert_array_equal(x, t)
    c.close()


@pytest.mark.parametrize("name", list(SETS))
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_scatter_matches_oracle(name, dtype):
    levels, coefs = SETS[name]()
    ts = _to_dev([np.full(W.shape_of(l), np.nan, dtype=dtype) for l in levels])
    c = sgh.Combination(ts, levels, coefs, graph=False)
    rng = np.random.default_rng(12)
    sp_host = rng.uniform(-1, 1, c.sparse_points).astype(dtype)
    c.scatter(torch.from_numpy(sp_host).cuda())
    refs = oracle.combi_scatter(sp_host.astype(np.float64), levels)
    for g, (got, ref) in enumerate(zip(_host(ts), refs)):
        np.testing.assert_array_equal(got.astype(np.float64), ref, err_msg="grid %d" % g)
    c.close()


def _check_reduce(xs, levels, coefs, ts, sp, dtype):
    """Every sparse point and every grid point within its own bound, from the
    point's actual contributors (tests/combi_bounds.py)."""
    x64 = [x.astype(np.float64) for x in xs]
    ref_grids, ref_sp = oracle.combi_round_trip(x64, levels, coefs)
    sp_tol, grid_tol = reduce_bounds(x64, levels, coefs, dtype, ref_grids)
    got_sp = sp.cpu().numpy().astype(np.float64)
    got = _host(ts)
    worst_sp = float(np.max(np.abs(got_sp - ref_sp) / sp_tol)) if sp_tol.size else 0.0
    worst_g = max((float(np.max(np.abs(g.astype(np.float64) - r) / t)) for g, r, t in zip(got, ref_grids, grid_tol)
                   if r.size), default=0.0)
    print("reduce %s: worst error / bound: sparse %.3f, grids %.3f" % (np.dtype(dtype).name, worst_sp, worst_g),
          flush=True)
    assert reduce_violations(got_sp, got, ref_sp, ref_grids, sp_tol, grid_tol) == (0, 0)


@pytest.mark.parametrize("name", list(SETS))
@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_reduce_matches_oracle_round_trip(name, dtype, graph):
    levels, coefs = SETS[name]()
    xs = W.combination_values(levels, seed=13, dtype=dtype)
    ts = _to_dev(xs)
    c = sgh.Combination(ts, levels, coefs, graph=graph)
    sp = c.new_sparse()
    c.reduce(sp)
    _check_reduce(xs, levels, coefs, ts, sp, dtype)
    c.close()


def test_reduce_graph_replays_with_eager_work_between():
    levels, coefs = W.combination_set(3, 7)
    xs = W.combination_values(levels, seed=14)
    originals = _to_dev(xs)
    ts = [o.clone() for o in originals]
    c = sgh.Combination(ts, levels, coefs, graph=True)
    sp = c.new_sparse()
    for rep in range(4):
        for t, o in zip(ts, originals):
            t.copy_(o)
        sp.fill_(float(rep))  # eager work on the stream between replays
        torch.cuda.synchronize()
        c.reduce(sp)
        _check_reduce(xs, levels, coefs, ts, sp, np.float64)
    c.close()


def test_reduce_is_a_projection():
    # combining an already combined set gives it back (up to rounding): the
    # sparse surpluses of the combined grids are the same sparse surpluses
    levels, coefs = W.combination_set(3, 6)
    xs = W.combination_values(levels, seed=15)
    ts = _to_dev(xs)
    c = sgh.Combination(ts, levels, coefs, graph=True)
    sp = c.new_sparse()
    c.reduce(sp)
    first = [t.clone() for t in ts]
    sp1 = sp.clone()
    c.reduce(sp)
    torch.cuda.synchronize()
    assert torch.max(torch.abs(sp - sp1)).item() <= 1e-13 * torch.max(torch.abs(sp1)).item()
    for a, b in zip(first, ts):
        assert torch.max(torch.abs(a - b)).item() <= 1e-13 * max(1.0, torch.max(torch.abs(a)).item())
    c.close()


def test_single_grid_set_is_identity():
    levels, coefs = [(5, 4, 3)], [1.0]
    xs = W.combination_values(levels, seed=16)
    ts = _to_dev(xs)
    c = sgh.Combination(ts, levels, coefs, graph=False)
    assert c.sparse_points == W.num_points(levels[0])
    sp = c.new_sparse()
    c.reduce(sp)
    got = _host(ts)[0]
    assert np.max(np.abs(got - xs[0])) <= 1e-14 * np.abs(xs[0]).max() * 10
    c.close()


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_set_data_repoints(graph):
    levels, coefs = W.combination_set(2, 6)
    xs_a = W.combination_values(levels, seed=17)
    xs_b = W.combination_values(levels, seed=18)
    ta, tb = _to_dev(xs_a), _to_dev(xs_b)
    c = sgh.Combination(ta, levels, coefs, graph=graph)
    sp = c.new_sparse()
    c.reduce(sp)
    _check_reduce(xs_a, levels, coefs, ta, sp, np.float64)
    c.set_data(tb)
    c.reduce(sp)
    _check_reduce(xs_b, levels, coefs, tb, sp, np.float64)
    # a second sparse buffer re-captures the graph
    sp2 = c.new_sparse()
    for t, x in zip(tb, xs_b):
        t.copy_(torch.from_numpy(x))
    c.reduce(sp2)
    _check_reduce(xs_b, levels, coefs, tb, sp2, np.float64)
    c.close()


def test_binding_rejects_bad_sparse_buffer():
    levels, coefs = W.combination_set(2, 4)
    ts = _to_dev(W.combination_values(levels, seed=19))
    c = sgh.Combination(ts, levels, coefs, graph=False)
    with pytest.raises(ValueError):
        c.gather(torch.zeros(c.sparse_points + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        c.gather(torch.zeros(c.sparse_points, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        c.gather(torch.zeros(c.sparse_points, dtype=torch.float64))
    with pytest.raises(sgh.SghError):
        sgh.Combination(ts + [torch.zeros(3, 3, dtype=torch.float32, device="cuda")],
                        levels + [(2, 2)], coefs + [1.0])
    c.close()
