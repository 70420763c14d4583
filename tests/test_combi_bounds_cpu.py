"""The per-point bounds of the reduce-step check (tests/combi_bounds.py) on the
CPU: the oracle's own result lies inside them, an error of a small fraction of
a bound passes, and planted mistakes of the kind the check exists to catch (a
contributor dropped from one sparse point's sum, a flipped coefficient, a grid
point whose scatter took a neighbour's value) fall outside them."""
import numpy as np
import pytest

import oracle
from combi_bounds import reduce_bounds, reduce_violations
from paper_1309_0392_amd import workloads as W


@pytest.fixture(scope="module")
def case():
    levels, coefs = W.combination_set(3, 6)
    xs = W.combination_values(levels, seed=31)
    ref_grids, ref_sp = oracle.combi_round_trip(xs, levels, coefs)
    bounds = {dt: reduce_bounds(xs, levels, coefs, dt, ref_grids) for dt in (np.float64, np.float32)}
    return levels, coefs, xs, ref_grids, ref_sp, bounds


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_oracle_result_and_small_noise_pass(case, dtype):
    levels, coefs, xs, ref_grids, ref_sp, bounds = case
    sp_tol, grid_tol = bounds[dtype]
    assert np.all(sp_tol > 0) and all(np.all(t > 0) for t in grid_tol)
    assert reduce_violations(ref_sp, ref_grids, ref_sp, ref_grids, sp_tol, grid_tol) == (0, 0)
    rng = np.random.default_rng(0)
    noisy_sp = ref_sp + 0.5 * sp_tol * rng.uniform(-1, 1, ref_sp.shape)
    noisy = [r + 0.5 * t * rng.uniform(-1, 1, r.shape) for r, t in zip(ref_grids, grid_tol)]
    assert reduce_violations(noisy_sp, noisy, ref_sp, ref_grids, sp_tol, grid_tol) == (0, 0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_dropped_contributor_is_caught(case, dtype):
    levels, coefs, xs, ref_grids, ref_sp, bounds = case
    sp_tol, grid_tol = bounds[dtype]
    hs = [oracle.hierarchize(x, l) for x, l in zip(xs, levels)]
    # the sum without grid 5 (a q = 0 grid): every sparse point it holds loses c_5 s_5(p)
    drop = list(coefs)
    drop[5] = 0.0
    bad_sp = oracle.combi_gather(hs, levels, drop)
    grids = [oracle.dehierarchize(b, l) for b, l in zip(oracle.combi_scatter(bad_sp, levels), levels)]
    n_sp, n_grid = reduce_violations(bad_sp, grids, ref_sp, ref_grids, sp_tol, grid_tol)
    assert n_sp > 0 and n_grid > 0


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_flipped_coefficient_is_caught(case, dtype):
    levels, coefs, xs, ref_grids, ref_sp, bounds = case
    sp_tol, grid_tol = bounds[dtype]
    hs = [oracle.hierarchize(x, l) for x, l in zip(xs, levels)]
    flip = list(coefs)
    flip[-1] = -flip[-1]
    bad_sp = oracle.combi_gather(hs, levels, flip)
    assert reduce_violations(bad_sp, ref_grids, ref_sp, ref_grids, sp_tol, grid_tol)[0] > 0


def test_one_wrong_grid_point_is_caught(case):
    levels, coefs, xs, ref_grids, ref_sp, bounds = case
    sp_tol, grid_tol = bounds[np.float32]
    grids = [r.copy() for r in ref_grids]
    g = grids[3]
    flat = g.reshape(-1)
    flat[7] = flat[8]  # one point took its neighbour's value
    assert reduce_violations(ref_sp, grids, ref_sp, ref_grids, sp_tol, grid_tol) == (0, 1)
