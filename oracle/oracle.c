/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the
 * hierarchization of the combination grids of the sparse grid combination
 * technique (P. Hupp, "Hierarchization for the Sparse Grid Combination
 * Technique", arXiv:1309.0392).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * Arithmetic is IEEE double precision, round-to-nearest, no fast-math.
 *
 * Conventions, all from the paper:
 *  - A combination grid is completely described by its level vector
 *    (l_1, ..., l_d); level 1 is a single grid point (Section 2, "The
 *    Combination Technique").  Hence axis k holds 2^{l_k} - 1 points.
 *  - The outermost points of a level have only one hierarchical
 *    predecessor (Section 3, text after Algorithm 1): the other one would lie
 *    on the boundary, which is not stored.  A missing predecessor contributes
 *    nothing.
 *  - Data is dense and row major with x_1 (axis 0 here) changing fastest
 *    (Section 3, "Unrolling and Vectorization").  The pole along axis k of a
 *    point therefore has stride prod_{j<k} (2^{l_j} - 1).
 *
 * Position convention used below: along a pole of level L the points carry
 * 1-based positions p = 1 .. 2^L - 1, stored at offset (p - 1) * stride.  A
 * point on 1-d level m (1 <= m <= L) sits at an odd multiple of the spacing
 * h = 2^(L-m); its left and right hierarchical predecessors are the nearest
 * coarser points p - h and p + h (binary-tree picture, Fig. 3 left).
 *
 * Parity status (see the test suite for the pins):
 *  - oracle_hierarchize: pinned (hat basis, linear reproduction, dense
 *    hat-evaluation inverse, sine closed form, axis-order invariance).
 *  - oracle_dehierarchize: pinned (inverse of the hat-evaluation matrix,
 *    round trips).
 *  - oracle_hierarchize_adjoint: pinned (dense transpose built from unit
 *    vectors, dot-product identity).
 *  - oracle_flops_eq1 / oracle_mults_reduced: pinned against brute-force
 *    counts of predecessor updates.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_DIM 16

/* Number of interior points of a 1-d grid of level L (level 1 = 1 point). */
static int64_t points_of_level(int L) { return ((int64_t)1 << L) - 1; }

/* 2^e as a double, exact for 0 <= e <= 62. */
static double pow2(int e) { return (double)((int64_t)1 << e); }

/* Total number of stored points of a grid: product of 2^{l_k} - 1. */
int64_t oracle_num_points(int d, const int *level)
{
    int64_t n = 1;
    for (int k = 0; k < d; ++k) n *= points_of_level(level[k]);
    return n;
}

/* Stride (in elements) of axis k: product of the point counts of the faster
 * axes, since axis 0 is the fastest-changing index. */
static int64_t axis_stride(int d, const int *level, int k)
{
    int64_t s = 1;
    (void)d;
    for (int j = 0; j < k; ++j) s *= points_of_level(level[j]);
    return s;
}

/* --- one 1-d pole -------------------------------------------------------
 * v points at pole position 1 (offset 0); position p lives at v[(p-1)*st].
 */

/* Algorithm 1, the two innermost loops: levels L down to 2; on each level
 * every point subtracts half of its left predecessor, then half of its right
 * predecessor.  The coarser predecessors have not been touched yet when they
 * are read, so they are still nodal values. */
static void pole_hierarchize(double *v, int64_t st, int L)
{
    const int64_t top = (int64_t)1 << L; /* position of the right boundary */
    for (int m = L; m >= 2; --m) {
        const int64_t h = (int64_t)1 << (L - m);
        for (int64_t p = h; p < top; p += 2 * h) { /* odd multiples of h */
            double *x = &v[(p - 1) * st];
            if (p - h >= 1) *x = *x - 0.5 * v[(p - h - 1) * st];
            if (p + h <= top - 1) *x = *x - 0.5 * v[(p + h - 1) * st];
        }
    }
}

/* Dehierarchization (the base change back to the nodal basis, Section 2,
 * "The Iterated Combination Technique"): the exact inverse of the loops
 * above.  Levels run from coarse to fine so that both predecessors already
 * hold nodal values when a point adds half of each of them back. */
static void pole_dehierarchize(double *v, int64_t st, int L)
{
    const int64_t top = (int64_t)1 << L;
    for (int m = 2; m <= L; ++m) {
        const int64_t h = (int64_t)1 << (L - m);
        for (int64_t p = h; p < top; p += 2 * h) {
            double *x = &v[(p - 1) * st];
            if (p - h >= 1) *x = *x + 0.5 * v[(p - h - 1) * st];
            if (p + h <= top - 1) *x = *x + 0.5 * v[(p + h - 1) * st];
        }
    }
}

/* Transpose of the hierarchization: every elementary update
 * "x[p] -= 0.5 * x[q]" of the forward loops becomes "x[q] -= 0.5 * x[p]",
 * and the whole sequence of updates is reversed: levels run from coarse to
 * fine, the points of a level from right to left, and inside a point the
 * right predecessor's update comes first.  When a level-m point is read it
 * has not been touched yet (only finer points update it, and they come
 * later). */
static void pole_adjoint(double *v, int64_t st, int L)
{
    const int64_t top = (int64_t)1 << L;
    for (int m = 2; m <= L; ++m) {
        const int64_t h = (int64_t)1 << (L - m);
        for (int64_t p = top - h; p >= h; p -= 2 * h) {
            const double xp = v[(p - 1) * st];
            if (p + h <= top - 1) v[(p + h - 1) * st] -= 0.5 * xp;
            if (p - h >= 1) v[(p - h - 1) * st] -= 0.5 * xp;
        }
    }
}

typedef void (*pole_fn)(double *, int64_t, int);

/* Second loop of Algorithm 1: split the grid into all 1-d poles in the
 * working direction k and apply fn to each. */
static void for_all_poles(double *x, int d, const int *level, int k, pole_fn fn)
{
    const int L = level[k];
    const int64_t n = points_of_level(L);
    const int64_t st = axis_stride(d, level, k);
    const int64_t total = oracle_num_points(d, level);
    const int64_t outer = total / (n * st);
    /* The poles are disjoint, so they may run on several threads: built with
     * OpenMP (the multi-core timing build) they are shared out statically;
     * the arithmetic of each pole is the same either way. */
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t o = 0; o < outer; ++o)
        for (int64_t s = 0; s < st; ++s)
            fn(x + o * n * st + s, st, L);
}

/* Threads the pole loops use: 1, or OpenMP's count in the multi-core build. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int check_args(const double *x, int d, const int *level)
{
    if (!x || !level || d < 1 || d > ORACLE_MAX_DIM) return -1;
    for (int k = 0; k < d; ++k)
        if (level[k] < 1 || level[k] > 30) return -1;
    return 0;
}

/* Algorithm 1: outer loop over the dimensions in the order 1..d. */
int oracle_hierarchize(double *x, int d, const int *level)
{
    if (check_args(x, d, level)) return -1;
    for (int k = 0; k < d; ++k) for_all_poles(x, d, level, k, pole_hierarchize);
    return 0;
}

/* One working direction only (the body of the outer loop of Algorithm 1). */
int oracle_hierarchize_axis(double *x, int d, const int *level, int axis)
{
    if (check_args(x, d, level) || axis < 0 || axis >= d) return -1;
    for_all_poles(x, d, level, axis, pole_hierarchize);
    return 0;
}

/* Inverse: the dimensions are undone in reverse order (they commute, so any
 * order is exact up to rounding; reverse order is the literal inverse of the
 * sequence). */
int oracle_dehierarchize(double *x, int d, const int *level)
{
    if (check_args(x, d, level)) return -1;
    for (int k = d - 1; k >= 0; --k) for_all_poles(x, d, level, k, pole_dehierarchize);
    return 0;
}

int oracle_dehierarchize_axis(double *x, int d, const int *level, int axis)
{
    if (check_args(x, d, level) || axis < 0 || axis >= d) return -1;
    for_all_poles(x, d, level, axis, pole_dehierarchize);
    return 0;
}

/* Transpose: the transposed per-dimension passes in reverse dimension
 * order. */
int oracle_hierarchize_adjoint(double *x, int d, const int *level)
{
    if (check_args(x, d, level)) return -1;
    for (int k = d - 1; k >= 0; --k) for_all_poles(x, d, level, k, pole_adjoint);
    return 0;
}

int oracle_hierarchize_adjoint_axis(double *x, int d, const int *level, int axis)
{
    if (check_args(x, d, level) || axis < 0 || axis >= d) return -1;
    for_all_poles(x, d, level, axis, pole_adjoint);
    return 0;
}

/* Flop count of Algorithm 1, Eq. (1) of Section 3 ("Flop Count"), in the
 * corrected reading: a pole of level L performs sum_{m=2..L} (2^m - 2)
 * predecessor updates (2^{m-1} points on level m, each with two predecessors
 * except the two outermost ones), i.e. 2^{L+1} - 2L - 2 updates of one
 * multiplication and one subtraction each; the number of poles in direction i
 * is the product of the other axes' point counts.  The printed formula has
 * 2^{l_i} in place of 2^{l_i+1}, which is negative for l_i <= 2. */
double oracle_flops_eq1(int d, const int *level)
{
    double f = 0.0;
    for (int i = 0; i < d; ++i) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j)
            if (j != i) prod *= (double)points_of_level(level[j]);
        const double Li = (double)level[i];
        f += (pow2(level[i] + 1) - 2.0 * Li - 2.0) * prod;
    }
    return 2.0 * f;
}

/* Multiplications of the reduced-operation variant (Section 3, after
 * Eq. (1)): a point with both predecessors adds them first and multiplies
 * once, so every point of levels 2..L costs exactly one multiplication:
 * 2^L - 2 per pole.  The additions stay at half of Eq. (1). */
double oracle_mults_reduced(int d, const int *level)
{
    double m = 0.0;
    for (int i = 0; i < d; ++i) {
        double prod = 1.0;
        for (int j = 0; j < d; ++j)
            if (j != i) prod *= (double)points_of_level(level[j]);
        m += (pow2(level[i]) - 2.0) * prod;
    }
    return m;
}

/* --- single output points ------------------------------------------------
 * For checks at full size, where running the whole oracle per test would be
 * too slow, these evaluate one output point directly.  pos[k] is the 1-based
 * position along axis k.  Each is the per-point reading of the whole-grid
 * routine above, derived in its comment, and the test suite checks it against
 * that routine on small grids.
 */

static int64_t offset_of(int d, const int *level, const int64_t *pos)
{
    int64_t off = 0, st = 1;
    for (int k = 0; k < d; ++k) {
        off += (pos[k] - 1) * st;
        st *= points_of_level(level[k]);
    }
    return off;
}

/* Spacing h of the point at position p of a level-L pole: p is an odd
 * multiple of h, and h = 2^(L-m) for its level m. */
static int64_t spacing_of(int64_t p)
{
    int64_t h = 1;
    while ((p & h) == 0) h <<= 1;
    return h;
}

/* Hierarchization at one point.  Within one pole, Algorithm 1 reads the
 * predecessors while they are still nodal, so one dimension's pass maps z to
 * z(p) - 0.5 z(p - h) - 0.5 z(p + h) (missing predecessors are skipped).
 * Composing the passes of dimensions 1..k gives the recursion below, which
 * applies the pass of dimension k to the result of dimensions 1..k-1. */
static double hier_point_rec(const double *x, int d, const int *level, int64_t *pos, int k)
{
    if (k < 0) return x[offset_of(d, level, pos)];
    const int64_t top = (int64_t)1 << level[k];
    const int64_t p = pos[k], h = spacing_of(p);
    double v = hier_point_rec(x, d, level, pos, k - 1);
    if (p - h >= 1) {
        pos[k] = p - h;
        v = v - 0.5 * hier_point_rec(x, d, level, pos, k - 1);
    }
    if (p + h <= top - 1) {
        pos[k] = p + h;
        v = v - 0.5 * hier_point_rec(x, d, level, pos, k - 1);
    }
    pos[k] = p;
    return v;
}

double oracle_hierarchize_point(const double *x, int d, const int *level, const int64_t *pos)
{
    int64_t q[ORACLE_MAX_DIM];
    for (int k = 0; k < d; ++k) q[k] = pos[k];
    return hier_point_rec(x, d, level, q, d - 1);
}

/* Dehierarchization at one point: the nodal value of the hierarchical
 * representation, i.e. the sum over all basis functions of surplus times the
 * tensor-product hat function evaluated at the point (Section 2, "Sparse
 * Grids": the hierarchical basis replaces the nodal basis).  Along one axis
 * the level-m' hat functions have half-width h' = 2^(L-m') and centres at odd
 * multiples of h'; at most one of them is nonzero at p, with value
 * 1 - |p - c| / h'.  Levels finer than the point's own level vanish there. */
static double dehier_point_rec(const double *s, int d, const int *level, int64_t *pos,
                               const int64_t *target, int k, double w)
{
    if (k < 0) return w * s[offset_of(d, level, pos)];
    const int L = level[k];
    const int64_t p = target[k];
    double acc = 0.0;
    for (int m = 1; m <= L; ++m) {
        const int64_t h = (int64_t)1 << (L - m);
        const int64_t c = (2 * (p / (2 * h)) + 1) * h; /* centre of the hat over p */
        const int64_t dist = p > c ? p - c : c - p;
        if (dist >= h) continue;                        /* p sits on a coarser node */
        const double phi = 1.0 - (double)dist / (double)h;
        pos[k] = c;
        acc += dehier_point_rec(s, d, level, pos, target, k - 1, w * phi);
    }
    pos[k] = target[k];
    return acc;
}

double oracle_dehierarchize_point(const double *s, int d, const int *level, const int64_t *pos)
{
    int64_t q[ORACLE_MAX_DIM];
    for (int k = 0; k < d; ++k) q[k] = pos[k];
    return dehier_point_rec(s, d, level, q, pos, d - 1, 1.0);
}

/* Transposed hierarchization at one point: (H^T g)(j) = sum_i H(i, j) g(i).
 * Along one axis, H(i, j) is 1 for i = j and -1/2 when j is a predecessor of
 * i; the points whose predecessor is j are j - h_m and j + h_m on every level
 * m finer than j's level (h_m = 2^(L-m)), and all of them are interior. */
static double adj_point_rec(const double *g, int d, const int *level, int64_t *pos,
                            const int64_t *target, int k)
{
    if (k < 0) return g[offset_of(d, level, pos)];
    const int L = level[k];
    const int64_t j = target[k], hj = spacing_of(j);
    double v = adj_point_rec(g, d, level, pos, target, k - 1);
    for (int64_t h = hj >> 1; h >= 1; h >>= 1) {
        pos[k] = j - h;
        v = v - 0.5 * adj_point_rec(g, d, level, pos, target, k - 1);
        pos[k] = j + h;
        v = v - 0.5 * adj_point_rec(g, d, level, pos, target, k - 1);
    }
    (void)L;
    pos[k] = j;
    return v;
}

double oracle_hierarchize_adjoint_point(const double *g, int d, const int *level, const int64_t *pos)
{
    int64_t q[ORACLE_MAX_DIM];
    for (int k = 0; k < d; ++k) q[k] = pos[k];
    return adj_point_rec(g, d, level, q, pos, d - 1);
}

/* --- combination technique: gather and scatter of surpluses ---------------
 *
 * Hierarchization is the preprocessing step of the combination technique's
 * communication phase (Section 2, "Hierarchization as preprocessing"): in the
 * hierarchical basis a point that a combination grid lacks has surplus zero,
 * so combining grids needs no interpolation.  The sparse grid's surplus at a
 * hierarchical point is the coefficient-weighted sum of the surpluses of every
 * combination grid that contains the point (Fig. 1: weights +1/-1 in 2-d).
 *
 * Sparse-grid storage: a list of hierarchical subspaces, each given by its
 * level vector m (point i of axis k sits at odd position (2 i + 1) on level
 * m_k, i = 0 .. 2^(m_k - 1) - 1) and stored densely with axis 0 fastest,
 * starting at offsets[s].  A grid point at 1-based position p on a level-L
 * axis has 1-d level m = L - log2(h), h its spacing (p an odd multiple of h),
 * and odd index p / h on that level.
 */

/* 1-d level and odd index of position p on an axis of level L. */
static void level_index(int64_t p, int L, int *m, int64_t *j)
{
    int lev = L;
    while (p % 2 == 0) { p /= 2; --lev; }
    *m = lev;
    *j = p;
}

/* Subspace of level vector m in the list (linear search), or -1. */
static int find_subspace(int d, const int *m, int nsub, const int *sub_levels)
{
    for (int s = 0; s < nsub; ++s) {
        int eq = 1;
        for (int k = 0; k < d && eq; ++k) eq = sub_levels[s * d + k] == m[k];
        if (eq) return s;
    }
    return -1;
}

/* Element of the sparse array holding the point (m, j). */
static int64_t sparse_index(int d, const int *m, const int64_t *j, const int64_t *offsets, int s)
{
    int64_t idx = 0, st = 1;
    for (int k = 0; k < d; ++k) {
        idx += ((j[k] - 1) / 2) * st;
        st *= (int64_t)1 << (m[k] - 1);
    }
    return offsets[s] + idx;
}

/* Visit every point of grid g: compute its hierarchical point and call back. */
typedef void (*combi_visit)(double *grid_val, double *sparse_val, double coef);

static int combi_walk(int ngrids, double *const *grids, const int *levels, const double *coefs, int d,
                      int nsub, const int *sub_levels, const int64_t *offsets, double *sparse, combi_visit fn)
{
    if (d < 1 || d > ORACLE_MAX_DIM) return -1;
    for (int g = 0; g < ngrids; ++g) {
        const int *L = levels + g * d;
        const int64_t N = oracle_num_points(d, L);
        int64_t pos[ORACLE_MAX_DIM], j[ORACLE_MAX_DIM];
        int m[ORACLE_MAX_DIM];
        for (int64_t e = 0; e < N; ++e) {
            int64_t r = e;
            for (int k = 0; k < d; ++k) {
                const int64_t nk = points_of_level(L[k]);
                pos[k] = r % nk + 1;
                r /= nk;
                level_index(pos[k], L[k], &m[k], &j[k]);
            }
            const int s = find_subspace(d, m, nsub, sub_levels);
            if (s < 0) return -2; /* the sparse grid lacks a point of this grid */
            fn(&grids[g][e], &sparse[sparse_index(d, m, j, offsets, s)], coefs ? coefs[g] : 1.0);
        }
    }
    return 0;
}

static void visit_gather(double *grid_val, double *sparse_val, double coef) { *sparse_val += coef * *grid_val; }
static void visit_scatter(double *grid_val, double *sparse_val, double coef)
{
    (void)coef;
    *grid_val = *sparse_val;
}

/* sparse = sum over grids, in list order, of coef * surplus (sparse is
 * zeroed first, sparse_size elements). */
int oracle_combi_gather(int ngrids, double *const *grids, const int *levels, const double *coefs, int d,
                        int nsub, const int *sub_levels, const int64_t *offsets, int64_t sparse_size,
                        double *sparse)
{
    for (int64_t i = 0; i < sparse_size; ++i) sparse[i] = 0.0;
    return combi_walk(ngrids, grids, levels, coefs, d, nsub, sub_levels, offsets, sparse, visit_gather);
}

/* Every grid point takes the sparse grid's surplus at its hierarchical point. */
int oracle_combi_scatter(int ngrids, double *const *grids, const int *levels, int d, int nsub,
                         const int *sub_levels, const int64_t *offsets, double *sparse)
{
    return combi_walk(ngrids, grids, levels, 0, d, nsub, sub_levels, offsets, sparse, visit_scatter);
}
