"""Per-point error bounds of the combination-technique reduce step
(hierarchize every grid, gather into the sparse grid, scatter back,
dehierarchize every grid), computed with the oracle from each point's actual
contributors.

Sparse point p (the grids g that hold it, coefficients c_g, surpluses s_g(p)):
  * each surplus carries the transform's tolerance, TOL * max|x_g|, weighted
    by |c_g| in the sum;
  * the product c_g * s_g(p) and the n(p) - 1 additions each round by at most
    one unit roundoff u of a partial sum bounded by sum_g |c_g| |s_g(p)|.
  So  |sp(p) - sp_ref(p)| <= TOL * sum_{g>p} |c_g| max|x_g|
                             + (n(p) + 1) u sum_{g>p} |c_g| |s_g(p)|.
Grid point q after the scatter and the inverse: its nodal value is a sum of
sparse surpluses with nonnegative hat weights (at most 1), so the sparse
errors propagate as  dehierarchize(scatter(bound))(q), computed exactly by the
oracle on the nonnegative bound; the inverse's own rounding adds TOL times the
larger of its input and output magnitudes, as in the transform tests.  Sums
over the contributors are taken with the oracle's gather on grids of
magnitudes (|c_g| as coefficients), so no bound is multiplied up by the number
of grids or by prod_k l_k."""
import numpy as np

import oracle

TOL = {np.float64: 1e-14, np.float32: 2e-6}
UNIT_ROUNDOFF = {np.float64: 2.0 ** -53, np.float32: 2.0 ** -24}


def reduce_bounds(xs64, levels, coefs, dtype, ref_grids=None):
    """Per-point tolerances (sparse array, list of grid arrays) of the reduce
    step on the FP64 inputs xs64, for results stored in `dtype`."""
    layout = oracle.sparse_layout(levels)
    acoef = [abs(float(c)) for c in coefs]
    tol, u = TOL[dtype], UNIT_ROUNDOFF[dtype]
    a = oracle.combi_gather([np.full(x.shape, np.abs(x).max() if x.size else 0.0) for x in xs64], levels, acoef,
                            layout)
    mags = [np.abs(oracle.hierarchize(x, l)) for x, l in zip(xs64, levels)]
    b = oracle.combi_gather(mags, levels, acoef, layout)
    n = oracle.combi_gather([np.ones(x.shape) for x in xs64], levels, [1.0] * len(levels), layout)
    sp_tol = tol * a + (n + 1.0) * u * b
    if ref_grids is None:
        ref_grids, _ = oracle.combi_round_trip(xs64, levels, coefs)
    scattered_bound = oracle.combi_scatter(sp_tol, levels, layout)
    scattered_mag = oracle.combi_scatter(np.abs(oracle.combi_gather(
        [oracle.hierarchize(x, l) for x, l in zip(xs64, levels)], levels, coefs, layout)), levels, layout)
    grid_tol = []
    for sb, sm, ref, l in zip(scattered_bound, scattered_mag, ref_grids, levels):
        own = tol * max(float(np.abs(sm).max()) if sm.size else 0.0, float(np.abs(ref).max()) if ref.size else 0.0)
        grid_tol.append(oracle.dehierarchize(sb, l) + own)
    return sp_tol, grid_tol


def reduce_violations(got_sp, got_grids, ref_sp, ref_grids, sp_tol, grid_tol):
    """Number of sparse points and grid points outside their bounds."""
    bad_sp = int(np.count_nonzero(np.abs(np.asarray(got_sp, dtype=np.float64) - ref_sp) > sp_tol))
    bad_grid = 0
    for got, ref, t in zip(got_grids, ref_grids, grid_tol):
        bad_grid += int(np.count_nonzero(np.abs(np.asarray(got, dtype=np.float64) - ref) > t))
    return bad_sp, bad_grid
