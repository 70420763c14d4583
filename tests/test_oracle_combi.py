"""Pins of the oracle's combination-technique gather / scatter.

The paper combines the combination grids' solutions by a weighted sum (Fig. 1)
and hierarchizes first so that missing points need no interpolation (Section 2,
"Hierarchization as preprocessing").  These checks tie the oracle's sparse-grid
gather and scatter to that nodal-basis definition and to identities of the
classical coefficients, without re-typing its loops."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1309_0392_amd import workloads as W

SETS = [(2, 4), (2, 5), (3, 3), (3, 4), (4, 3)]


@pytest.mark.parametrize("d,n", SETS + [(4, 10)])
def test_coefficients_sum_to_one_on_every_subspace(d, n):
    """sum of c_l over the grids l >= m is 1 for every subspace m of the sparse grid."""
    lv, coef = W.combination_set(d, n)
    sub, _, _ = oracle.sparse_layout(lv)
    L = np.array(lv)
    C = np.array(coef)
    for m in sub:
        assert C[np.all(L >= m, axis=1)].sum() == 1, m
    assert all(sum(m) <= n + d - 1 for m in sub)


def test_layout_order_and_size():
    lv, _ = W.combination_set(4, 10)
    sub, off, total = oracle.sparse_layout(lv)
    assert len(sub) == 715 and total == 178177       # all m >= 1 with |m|_1 <= 13
    keys = [(int(m.sum()), tuple(int(v) for v in m)) for m in sub]
    assert keys == sorted(keys)
    assert off[0] == 0 and np.all(np.diff(off) == (1 << (sub[:-1].sum(axis=1) - 4)))


def full_grid_function(n, d, seed):
    """An exactly representable function: random multiples of 1/16 on the full level-(n..n)
    grid, of which every grid of the set is a subgrid."""
    rng = np.random.default_rng(seed)
    return rng.integers(-64, 65, size=W.shape_of((n,) * d)) / 16.0


def sample(full, n, levels):
    """Values of the full level-(n..n) grid at the points of a coarser grid."""
    sl = tuple(slice((1 << (n - l)) - 1, None, 1 << (n - l)) for l in reversed(levels))
    return np.ascontiguousarray(full[sl])


@pytest.mark.parametrize("d,n", SETS)
def test_gather_of_one_function_gives_its_surpluses(d, n):
    """All grids sample one function: the gathered sparse surplus at (m, j) is that function's
    surplus there (coefficients sum to 1), equal to the surplus in the full grid."""
    lv, coef = W.combination_set(d, n)
    f = full_grid_function(n, d, 1)
    sf = oracle.hierarchize(f, (n,) * d)
    hs = [oracle.hierarchize(sample(f, n, l), l) for l in lv]
    sub, off, total = oracle.sparse_layout(lv)
    sp = oracle.combi_gather(hs, lv, coef)
    for s, m in enumerate(sub):
        for local, js in enumerate(itertools.product(*[range(1 << (mk - 1)) for mk in reversed(m)])):
            j = [2 * i + 1 for i in reversed(js)]            # odd index per axis, axis 0 first
            pos = [jk << (n - mk) for jk, mk in zip(j, m)]   # position in the full grid
            assert sp[off[s] + local] == sf[tuple(p - 1 for p in reversed(pos))]


@pytest.mark.parametrize("d,n", SETS)
def test_scatter_of_unit_surplus(d, n):
    lv, coef = W.combination_set(d, n)
    sub, off, total = oracle.sparse_layout(lv)
    rng = np.random.default_rng(2)
    for _ in range(5):
        s = int(rng.integers(len(sub)))
        m = sub[s]
        local = int(rng.integers(1 << int(m.sum() - d)))
        sp = np.zeros(total)
        sp[off[s] + local] = 1.0
        grids = oracle.combi_scatter(sp, lv)
        # odd index per axis from the local index (axis 0 fastest)
        j, r = [], local
        for mk in m:
            j.append(2 * (r % (1 << (mk - 1))) + 1)
            r //= 1 << (mk - 1)
        for g, l in zip(grids, lv):
            if np.all(np.array(l) >= m):
                pos = [jk << (lk - mk) for jk, lk, mk in zip(j, l, m)]
                expect = np.zeros_like(g)
                expect[tuple(p - 1 for p in reversed(pos))] = 1.0
                assert np.array_equal(g, expect)
            else:
                assert not g.any()
        # and gathering it back gives the unit surplus (coefficients sum to 1)
        assert np.array_equal(oracle.combi_gather(grids, lv, coef), sp)


def multilinear(values, levels, points):
    """Piecewise multilinear interpolant of grid data (zero boundary) at points in [0,1]^d."""
    d = len(levels)
    padded = np.pad(values, 1)  # zero boundary on every side
    out = np.zeros(len(points))
    for r, x in enumerate(points):
        acc = 0.0
        base, frac = [], []
        for k in range(d):
            t = x[k] * (1 << levels[k])
            i = min(int(np.floor(t)), (1 << levels[k]) - 1)
            base.append(i)
            frac.append(t - i)
        for corner in itertools.product((0, 1), repeat=d):
            w = 1.0
            idx = []
            for k in range(d):
                w *= frac[k] if corner[k] else 1.0 - frac[k]
                idx.append(base[k] + corner[k])
            acc += w * padded[tuple(reversed(idx))]
        out[r] = acc
    return out


@pytest.mark.parametrize("d,n", [(2, 4), (2, 5), (3, 3)])
def test_round_trip_equals_nodal_combination_formula(d, n):
    """hierarchize -> gather -> scatter -> dehierarchize puts on every grid the combined
    solution sum_l c_l u_l (u_l the multilinear interpolant of grid l's data), sampled at
    that grid's points: the combination formula of Fig. 1 evaluated in the nodal basis."""
    lv, coef = W.combination_set(d, n)
    rng = np.random.default_rng(3)
    xs = [rng.integers(-32, 33, size=W.shape_of(l)) / 8.0 for l in lv]
    out, _ = oracle.combi_round_trip(xs, lv, coef)
    for target, l in zip(out, lv):
        pts = list(itertools.product(*[np.arange(1, 1 << lk) / float(1 << lk) for lk in l]))
        combined = sum(c * multilinear(x, lsrc, pts) for c, x, lsrc in zip(coef, xs, lv))
        got = np.array([target[tuple(int(round(p * (1 << lk))) - 1 for p, lk in reversed(list(zip(pt, l))))]
                        for pt in pts])
        assert np.max(np.abs(got - combined)) <= 1e-12


@pytest.mark.parametrize("d,n", [(2, 5), (3, 4)])
def test_round_trip_of_one_function_is_identity(d, n):
    lv, coef = W.combination_set(d, n)
    f = full_grid_function(n, d, 4)
    xs = [sample(f, n, l) for l in lv]
    out, _ = oracle.combi_round_trip(xs, lv, coef)
    for a, b in zip(out, xs):
        assert np.array_equal(a, b)
