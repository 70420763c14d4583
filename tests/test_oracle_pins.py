"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types the oracle's loops: each compares it with an
independent description of the same map (hierarchical hat basis, piecewise
linear reproduction, tensor-product structure from a per-point predecessor
rule, closed forms, brute-force counts).  A dropped term, a wrong sign, a
swapped predecessor or a transposed operand in the oracle fails at least one.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_1309_0392_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers ---
def lowbit(p: int) -> int:
    return p & -p


def hat_value(level_m: int, index_j: int, x: float) -> float:
    """Hierarchical hat of level m and odd index j at coordinate x (exact for dyadic x)."""
    return max(0.0, 1.0 - abs(x * (1 << level_m) - index_j))


def grid_coords(levels):
    """Coordinates per grid axis: p / 2^l for p = 1..2^l-1."""
    return [np.arange(1, 1 << l) / float(1 << l) for l in levels]


def sample_tensor(levels, per_axis_fns):
    """Array of prod_k f_k(x_k) over the grid (numpy layout: axis 0 last)."""
    d = len(levels)
    out = np.ones(W.shape_of(levels))
    for k, (l, f) in enumerate(zip(levels, per_axis_fns)):
        v = np.array([f(x) for x in grid_coords([l])[0]])
        view = [1] * d
        view[d - 1 - k] = v.size
        out = out * v.reshape(view)
    return out


def point_level(p: int, L: int) -> int:
    """1-d level of position p on a level-L pole (level 1 = root)."""
    return L - (lowbit(p).bit_length() - 1)


def dense(fn, levels):
    """Matrix of the linear map fn on a grid, built column by column from unit vectors."""
    n = W.num_points(levels)
    shape = W.shape_of(levels)
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(fn(e.reshape(shape), levels).reshape(-1))
    return np.stack(cols, axis=1)


def one_d_from_predecessor_rule(L: int) -> np.ndarray:
    """1-d hierarchization matrix from the per-point rule s_p = x_p - x_{p-lb}/2 - x_{p+lb}/2."""
    n = (1 << L) - 1
    H = np.eye(n)
    for p in range(1, n + 1):
        b = lowbit(p)
        if p - b >= 1:
            H[p - 1, p - b - 1] = -0.5
        if p + b <= n:
            H[p - 1, p + b - 1] = -0.5
    return H


def hat_evaluation_matrix(levels) -> np.ndarray:
    """Phi[i, a] = hierarchical hat of grid point a evaluated at grid point i."""
    per_axis = []
    for L in levels:
        n = (1 << L) - 1
        P = np.zeros((n, n))
        for a in range(1, n + 1):
            m = point_level(a, L)
            j = a >> (L - m)  # odd index of a on its own level
            for i in range(1, n + 1):
                P[i - 1, a - 1] = hat_value(m, j, i / float(1 << L))
        per_axis.append(P)
    M = np.ones((1, 1))
    for P in per_axis:  # flat index = p0 + n0*p1 + ... -> kron(P_{d-1}, ..., P_0)
        M = np.kron(P, M)
    return M


TINY = [(1,), (2,), (3,), (4,), (3, 2), (2, 3), (2, 2, 2), (1, 3), (3, 1, 2), (2, 1, 1, 2)]


# ------------------------------------------------------- basis functions ---
@pytest.mark.parametrize("levels", [(5,), (4, 3), (3, 3, 2), (2, 3, 1, 2), (6, 5)])
def test_hat_basis_gives_single_unit_surplus(levels):
    """A sampled tensor-product hat is one hierarchical basis function: exactly one surplus 1."""
    rng = np.random.default_rng(11)
    for _ in range(12):
        m = [int(rng.integers(1, l + 1)) for l in levels]
        j = [int(2 * rng.integers(0, 1 << (mk - 1)) + 1) for mk in m]
        fns = [lambda x, mk=mk, jk=jk: hat_value(mk, jk, x) for mk, jk in zip(m, j)]
        x = sample_tensor(levels, fns)
        s = oracle.hierarchize(x, levels)
        expect = np.zeros_like(x)
        pos = tuple(jk << (l - mk) for l, mk, jk in zip(levels, m, j))  # 1-based, axis order
        expect[tuple(p - 1 for p in reversed(pos))] = 1.0
        assert np.array_equal(s, expect), (levels, m, j)
        # and the inverse maps the unit surplus back to the samples, exactly
        assert np.array_equal(oracle.dehierarchize(expect, levels), x)


@pytest.mark.parametrize("levels,coarse", [((6,), (3,)), ((5, 4), (3, 2)), ((4, 4, 3), (2, 3, 1)),
                                           ((3, 5), (3, 1))])
def test_linear_on_coarser_grid_has_zero_fine_surpluses(levels, coarse):
    """A piecewise (multi)linear function on a coarser grid has zero surplus on every finer level,
    and its coarse surpluses equal those of the coarse grid alone."""
    rng = np.random.default_rng(5)
    vc = rng.integers(-64, 65, size=W.shape_of(coarse)) / 16.0  # dyadic nodal values
    # nodal (piecewise linear) hat of level lc centred at node c: max(0, 1 - |x 2^lc - c|)
    x = np.zeros(W.shape_of(levels))
    for cidx in itertools.product(*[range(1, 1 << lc) for lc in coarse]):
        fns = [lambda t, lc=lc, c=c: max(0.0, 1.0 - abs(t * (1 << lc) - c)) for lc, c in zip(coarse, cidx)]
        x += vc[tuple(c - 1 for c in reversed(cidx))] * sample_tensor(levels, fns)
    s = oracle.hierarchize(x, levels)
    sc = oracle.hierarchize(vc, coarse)
    for flat, val in np.ndenumerate(s):
        pos = list(reversed([i + 1 for i in flat]))  # 1-based, grid axis order
        lv = [point_level(p, L) for p, L in zip(pos, levels)]
        if any(m > c for m, c in zip(lv, coarse)):
            assert val == 0.0, (pos, val)
        else:
            cpos = [p >> (L - c) for p, L, c in zip(pos, levels, coarse)]
            assert val == sc[tuple(c - 1 for c in reversed(cpos))]


# ------------------------------------------------------ dense structure ---
@pytest.mark.parametrize("levels", TINY)
def test_dense_hierarchization_inverts_hat_evaluation(levels):
    """Hierarchization is the base change nodal -> hierarchical: H @ Phi = I and dehier == Phi."""
    H = dense(oracle.hierarchize, levels)
    D = dense(oracle.dehierarchize, levels)
    Phi = hat_evaluation_matrix(levels)
    n = H.shape[0]
    assert np.array_equal(D, Phi)
    assert np.allclose(H @ Phi, np.eye(n), rtol=0, atol=1e-15)
    assert np.allclose(Phi @ H, np.eye(n), rtol=0, atol=1e-15)


@pytest.mark.parametrize("levels", TINY)
def test_dense_hierarchization_is_kronecker_of_predecessor_rule(levels):
    H = dense(oracle.hierarchize, levels)
    K = np.ones((1, 1))
    for L in levels:
        K = np.kron(one_d_from_predecessor_rule(L), K)
    assert np.array_equal(H, K)


@pytest.mark.parametrize("levels", TINY)
def test_dense_adjoint_is_transpose(levels):
    H = dense(oracle.hierarchize, levels)
    A = dense(oracle.hierarchize_adjoint, levels)
    assert np.array_equal(A, H.T)


@pytest.mark.parametrize("levels", [(3,), (2, 3), (3, 2, 2)])
def test_per_axis_routines_compose(levels):
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, W.shape_of(levels))
    for name, axis_fn, full in (("h", oracle.hierarchize_axis, oracle.hierarchize),
                                ("d", oracle.dehierarchize_axis, oracle.dehierarchize),
                                ("a", oracle.hierarchize_adjoint_axis, oracle.hierarchize_adjoint)):
        y = x.copy()
        for k in range(len(levels)):
            y = axis_fn(y, levels, k)
        assert np.allclose(y, full(x, levels), rtol=0, atol=1e-15), name


def test_bfs_order_is_unit_lower_triangular():
    """In the BFS layout of Fig. 3 (levels coarse to fine) the 1-d map is unit lower triangular."""
    with open(os.path.join(GOLDEN, "bfs_layout_level3.txt")) as f:
        seq = [int(t) for line in f if not line.startswith("#") for t in line.split()]
    L = 3
    assert sorted(seq) == seq and [seq.count(m) for m in (1, 2, 3)] == [1, 2, 4]
    positions = sorted(range(1, 1 << L), key=lambda p: (point_level(p, L), p))
    assert [point_level(p, L) for p in positions] == seq
    H = dense(oracle.hierarchize, (L,))
    perm = [p - 1 for p in positions]
    B = H[np.ix_(perm, perm)]
    assert np.array_equal(np.triu(B, 1), np.zeros_like(B))
    assert np.array_equal(np.diag(B), np.ones(len(perm)))
    for L in range(1, 8):  # every level: BFS-ordered matrix is unit lower triangular (det 1)
        H = dense(oracle.hierarchize, (L,))
        perm = [p - 1 for p in sorted(range(1, 1 << L), key=lambda p: (point_level(p, L), p))]
        B = H[np.ix_(perm, perm)]
        assert np.array_equal(np.triu(B, 1), np.zeros_like(B)) and np.all(np.diag(B) == 1.0)


# ------------------------------------------------------ closed forms etc ---
@pytest.mark.parametrize("levels", [(7,), (6, 5), (5, 4, 4), (4, 3, 3, 3)])
def test_sine_product_closed_form(levels):
    """f = prod sin(pi x_k): surplus = prod_k 2 sin(pi x_k) sin^2(pi h_k / 2), h_k = parent distance.

    From sin(a-h) + sin(a+h) = 2 sin(a) cos(h); the zero boundary is sin(0) = sin(pi) = 0."""
    x = W.sine_plus_noise(levels, seed=0, noise=0.0)
    s = oracle.hierarchize(x, levels)
    fns = []
    for L in levels:
        vals = {}
        for p in range(1, 1 << L):
            h = lowbit(p) / float(1 << L)
            vals[p / float(1 << L)] = 2.0 * np.sin(np.pi * p / (1 << L)) * np.sin(np.pi * h / 2.0) ** 2
        fns.append(lambda t, vals=vals: vals[t])
    expect = sample_tensor(levels, fns)
    assert np.max(np.abs(s - expect)) <= 4e-16 * len(levels)


@pytest.mark.parametrize("levels", [(8,), (5, 4), (3, 4, 3), (2, 3, 2, 3), (1, 4, 1)])
def test_round_trips(levels):
    x = W.uniform(levels, 7)
    assert np.max(np.abs(oracle.dehierarchize(oracle.hierarchize(x, levels), levels) - x)) <= 1e-14
    assert np.max(np.abs(oracle.hierarchize(oracle.dehierarchize(x, levels), levels) - x)) <= 1e-14


@pytest.mark.parametrize("levels", [(4, 3, 2), (2, 5), (3, 2, 3, 2)])
def test_axis_order_invariance(levels):
    """Permuting the grid axes (data and level vector) and permuting back leaves the result."""
    x = W.uniform(levels, 9)
    ref = {"h": oracle.hierarchize(x, levels), "d": oracle.dehierarchize(x, levels),
           "a": oracle.hierarchize_adjoint(x, levels)}
    d = len(levels)
    for perm in itertools.permutations(range(d)):
        if perm == tuple(range(d)):
            continue
        lv = [levels[k] for k in perm]  # new grid axis i is old axis perm[i]
        # numpy axis of grid axis k is d-1-k
        np_axes = [d - 1 - perm[d - 1 - a] for a in range(d)]
        xp = np.ascontiguousarray(np.transpose(x, np_axes))
        inv = np.argsort(np_axes)
        for key, fn in (("h", oracle.hierarchize), ("d", oracle.dehierarchize), ("a", oracle.hierarchize_adjoint)):
            y = np.transpose(fn(xp, lv), inv)
            assert np.max(np.abs(y - ref[key])) <= 1e-14 * max(1.0, np.max(np.abs(ref[key]))), (perm, key)


@pytest.mark.parametrize("levels", [(6,), (4, 3), (3, 3, 2)])
def test_dot_product_identity(levels):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(W.shape_of(levels))
    y = rng.standard_normal(W.shape_of(levels))
    lhs = np.sum(oracle.hierarchize(x, levels) * y)
    rhs = np.sum(x * oracle.hierarchize_adjoint(y, levels))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("levels", [(5,), (3, 4), (3, 2, 3), (2, 2, 1, 3)])
def test_point_evaluators_match_whole_grid(levels):
    x = W.uniform(levels, 2)
    pos = np.array(list(itertools.product(*[range(1, 1 << l) for l in reversed(levels)])))[:, ::-1]
    for op, full in (("hierarchize", oracle.hierarchize), ("dehierarchize", oracle.dehierarchize),
                     ("adjoint", oracle.hierarchize_adjoint)):
        ref = full(x, levels)
        got = oracle.point(op, x, levels, pos)
        want = np.array([ref[tuple(p - 1 for p in reversed(r))] for r in pos])
        assert np.max(np.abs(got - want)) <= 1e-14, op


# --------------------------------------------------------- flop counts ---
def brute_force_updates(levels) -> int:
    """Predecessor updates of Algorithm 1, counted point by point with the lowbit rule."""
    total = 0
    for k, L in enumerate(levels):
        n = (1 << L) - 1
        per_pole = 0
        for p in range(1, n + 1):
            b = lowbit(p)
            per_pole += (p - b >= 1) + (p + b <= n)
        poles = 1
        for j, Lj in enumerate(levels):
            if j != k:
                poles *= (1 << Lj) - 1
        total += per_pole * poles
    return total


def test_flop_count_eq1_corrected():
    # one pole: 0, 2, 8, 22, 52, 114, 240 predecessor updates for l = 1..7
    assert [brute_force_updates((L,)) for L in range(1, 8)] == [0, 2, 8, 22, 52, 114, 240]
    for levels in [(L,) for L in range(1, 12)] + [(5, 5), (3, 2), (2, 3, 4), (1, 1, 5), (4, 4, 4, 2)]:
        assert oracle.flops_eq1(levels) == 2 * brute_force_updates(levels), levels
        # every point on levels >= 2 costs one multiplication in the reduced-op form
        poles_points = sum(((1 << L) - 2) * np.prod([(1 << Lj) - 1 for j, Lj in enumerate(levels) if j != k])
                           for k, L in enumerate(levels))
        assert oracle.mults_reduced(levels) == poles_points
    # The printed form, with 2^{l_i} instead of 2^{l_i+1}, would give negative counts:
    printed = lambda L: 2 * ((1 << L) - 2 * L - 2)
    assert printed(1) < 0 and printed(2) < 0
    # "roughly twice as many additions as multiplications" (A = F/2, M as printed) holds
    for L in range(8, 16):
        ratio = (oracle.flops_eq1((L,)) / 2) / oracle.mults_reduced((L,))
        assert 1.9 <= ratio <= 2.0


def test_workload_flop_counts():
    assert oracle.flops_eq1(W.SMALL_2D) == 6448
    assert oracle.flops_eq1(W.ANISO_3D) == 1568292744
    assert oracle.flops_eq1(W.ANISO_5D) == 2045869056
    lv, _ = W.combination_set()
    assert sum(oracle.flops_eq1(l) for l in lv) == 7707152


def test_size_rule():
    """|l|_1 = 27 is about 1 GB of doubles, and the size halves per level-sum step."""
    for levels in [(27,), (14, 13), (9, 9, 9), (7, 7, 7, 6)]:
        gib = oracle.num_points(levels) * 8 / 2 ** 30
        assert 0.9 <= gib <= 1.0, levels
        half = list(levels)
        half[0] -= 1
        r = oracle.num_points(half) / oracle.num_points(levels)
        assert 0.49 <= r <= 0.51


@pytest.mark.parametrize("levels", [(1,), (9,), (5, 5), (3, 6, 2), (2, 2, 2, 2, 3), (7, 1, 4)])
def test_threaded_build_matches_serial(levels):
    """The OpenMP build splits the poles of one direction across threads and
    runs each pole's loop unchanged, so every transform equals the serial
    build bit for bit (in place and on copies)."""
    x = W.uniform(levels, [17, sum(levels)])
    for f in (oracle.hierarchize, oracle.dehierarchize, oracle.hierarchize_adjoint):
        a = f(x, levels)
        b = f(x, levels, threads=True)
        assert np.array_equal(a, b), (f.__name__, levels)
    for f in (oracle.hierarchize_inplace, oracle.hierarchize_adjoint_inplace):
        a = x.copy()
        b = x.copy()
        f(a, levels)
        f(b, levels, threads=True)
        assert np.array_equal(a, b), (f.__name__, levels)
    assert oracle.num_threads(True) >= 1
