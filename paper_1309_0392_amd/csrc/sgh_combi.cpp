// Combination technique on the GPU: the sparse-grid layout of a combination
// set, gather / scatter of hierarchical surpluses, and one step of the
// iterated combination technique without the solver (hierarchize, gather,
// scatter, dehierarchize) captured as one HIP graph.  C ABI in include/sgh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "sgh.h"
#include "sgh_internal.h"

namespace sgh {
namespace {

int cfail(int code, const char *msg) { return report_error(code, msg); }

constexpr int64_t kMaxTable = int64_t(1) << 26;

}  // namespace
}  // namespace sgh

struct sgh_combi {
    int d = 0;
    int dtype = SGH_F64;
    std::vector<sgh_grid> grids;
    std::vector<double> coefs;
    std::vector<int32_t> sub_levels;   // nsub * d
    std::vector<int64_t> sub_offsets;  // nsub
    int64_t total = 0;
    int64_t tstride[SGH_MAX_DIM] = {};
    // device state
    sgh::CombiGrid *d_grids = nullptr;
    int32_t *d_sub_levels = nullptr;
    int64_t *d_sub_offsets = nullptr;
    int32_t *d_cbegin = nullptr;
    std::vector<int32_t> csub, cgrid;  // subspace and grid of each contribution
    int64_t *d_caddr = nullptr;
    int64_t *d_cmul = nullptr;
    double *d_ccoef = nullptr;
    int32_t fast32 = 0;
    int64_t *d_table = nullptr;
    sgh::CombiUnit *d_gunits = nullptr;
    sgh::CombiUnit *d_sunits = nullptr;
    int32_t ngunits = 0, nsunits = 0;
    sgh_plan *hier = nullptr;
    sgh_plan *dehier = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_sparse = nullptr;
    uint32_t flags = 0;
};

namespace sgh {
namespace {

void combi_free(sgh_combi *c) {
    for (void *p : {static_cast<void *>(c->d_grids), static_cast<void *>(c->d_sub_levels),
                    static_cast<void *>(c->d_sub_offsets), static_cast<void *>(c->d_cbegin),
                    static_cast<void *>(c->d_caddr), static_cast<void *>(c->d_cmul), static_cast<void *>(c->d_ccoef), static_cast<void *>(c->d_table),
                    static_cast<void *>(c->d_gunits), static_cast<void *>(c->d_sunits)})
        if (p) (void)hipFree(p);
    if (c->hier) sgh_plan_destroy(c->hier);
    if (c->dehier) sgh_plan_destroy(c->dehier);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

template <typename V>
hipError_t upload(V **dst, const std::vector<V> &src) {
    if (*dst) {
        (void)hipFree(*dst);
        *dst = nullptr;
    }
    const size_t bytes = std::max<size_t>(1, src.size()) * sizeof(V);
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
    return e;
}

// x / n as a multiply and a shift for 0 <= x < 2^31: with s = ceil(log2 n)
// and magic = floor(2^(32+s) / n) + 1 < 2^33, the error of x * magic / 2^(32+s)
// against x / n is below x / 2^(32+s) < 2^-(s+1) <= 1 / (2n), so the floor is exact.
void division_magic(int64_t n, uint64_t *magic, int32_t *shift) {
    int sh = 0;
    while ((int64_t(1) << sh) < n) ++sh;
    *magic = static_cast<uint64_t>((static_cast<unsigned __int128>(1) << (32 + sh)) / static_cast<uint64_t>(n)) + 1;
    *shift = 32 + sh;
}

std::vector<CombiGrid> grid_table(sgh_combi &c) {
    std::vector<CombiGrid> out;
    c.fast32 = 1;
    for (const auto &g : c.grids) {
        CombiGrid cg{};
        cg.data = g.data;
        int64_t st = 1;
        for (int k = 0; k < c.d; ++k) {
            cg.L[k] = g.level[k];
            cg.n[k] = (int64_t(1) << g.level[k]) - 1;
            cg.st[k] = st;
            division_magic(cg.n[k], &cg.magic[k], &cg.mshift[k]);
            st *= cg.n[k];
        }
        if (st >= (int64_t(1) << 31)) c.fast32 = 0;
        out.push_back(cg);
    }
    return out;
}

// Per contribution (subspace m, grid g): the grid's base address shifted by
// -sum_k st_k elements, and the element step 2^(L_k - m_k) st_k per odd index
// along axis k, so that the point with odd indices j sits at
// base + sum_k j_k * step_k.
hipError_t upload_contrib(sgh_combi *c) {
    const int d = c->d;
    const int64_t esize = c->dtype == SGH_F64 ? 8 : 4;
    std::vector<int64_t> addr(c->cgrid.size()), mul(c->cgrid.size() * static_cast<size_t>(d));
    for (size_t i = 0; i < c->cgrid.size(); ++i) {
        const sgh_grid &g = c->grids[static_cast<size_t>(c->cgrid[i])];
        const int32_t *m = &c->sub_levels[static_cast<size_t>(c->csub[i]) * static_cast<size_t>(d)];
        int64_t st = 1, sst = 0;
        for (int k = 0; k < d; ++k) {
            mul[i * static_cast<size_t>(d) + static_cast<size_t>(k)] = (int64_t(1) << (g.level[k] - m[k])) * st;
            sst += st;
            st *= (int64_t(1) << g.level[k]) - 1;
        }
        addr[i] = static_cast<int64_t>(reinterpret_cast<uintptr_t>(g.data)) - sst * esize;
    }
    hipError_t e = upload(&c->d_caddr, addr);
    if (e == hipSuccess) e = upload(&c->d_cmul, mul);
    return e;
}

CombiLaunch launch_of(const sgh_combi &c, bool gather, void *sparse) {
    CombiLaunch p{};
    p.d = c.d;
    p.nunits = gather ? c.ngunits : c.nsunits;
    p.grids = c.d_grids;
    p.sub_levels = c.d_sub_levels;
    p.sub_offsets = c.d_sub_offsets;
    p.contrib_begin = c.d_cbegin;
    p.contrib_addr = c.d_caddr;
    p.contrib_mul = c.d_cmul;
    p.contrib_coef = c.d_ccoef;
    p.fast32 = c.fast32;
    p.table = c.d_table;
    for (int k = 0; k < SGH_MAX_DIM; ++k) p.tstride[k] = c.tstride[k];
    p.units = gather ? c.d_gunits : c.d_sunits;
    p.sparse = sparse;
    return p;
}

hipError_t do_gather(const sgh_combi &c, void *sparse, hipStream_t s) {
    LaunchTimer t(c.dtype == SGH_F64 ? "combi_f64_gather" : "combi_f32_gather", s);
    const CombiLaunch p = launch_of(c, true, sparse);
    return c.dtype == SGH_F64 ? launch_combi_gather_f64(p, s) : launch_combi_gather_f32(p, s);
}

hipError_t do_scatter(const sgh_combi &c, const void *sparse, hipStream_t s) {
    LaunchTimer t(c.dtype == SGH_F64 ? "combi_f64_scatter" : "combi_f32_scatter", s);
    const CombiLaunch p = launch_of(c, false, const_cast<void *>(sparse));
    return c.dtype == SGH_F64 ? launch_combi_scatter_f64(p, s) : launch_combi_scatter_f32(p, s);
}

int64_t norm1(const std::vector<int32_t> &m) {
    int64_t s = 0;
    for (int v : m) s += v;
    return s;
}

// Subspaces of the sparse grid of a level set: every level vector m >= 1
// below some grid's levels, ordered by |m|_1, then lexicographically (axis 0
// compared first).
int subspaces_of(const sgh_grid *grids, int n, std::vector<std::vector<int32_t>> &order) {
    const int d = grids[0].dim;
    std::set<std::vector<int32_t>> subs;
    for (int g = 0; g < n; ++g) {
        std::vector<int32_t> m(static_cast<size_t>(d), 1);
        for (;;) {
            subs.insert(m);
            int k = 0;
            while (k < d && m[static_cast<size_t>(k)] == grids[g].level[k]) m[static_cast<size_t>(k++)] = 1;
            if (k == d) break;
            ++m[static_cast<size_t>(k)];
            if (subs.size() > (size_t(1) << 22)) return cfail(SGH_ERR_UNSUPPORTED, "too many subspaces");
        }
    }
    order.assign(subs.begin(), subs.end());
    std::stable_sort(order.begin(), order.end(), [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
        const int64_t na = norm1(a), nb = norm1(b);
        if (na != nb) return na < nb;
        return a < b;
    });
    return SGH_OK;
}

int check_set(const sgh_grid *grids, int32_t n) {
    if (n < 1 || !grids) return cfail(SGH_ERR_ARG, "need at least one grid");
    int rc = sgh_validate(grids, n);
    if (rc) return rc;
    for (int i = 1; i < n; ++i)
        if (grids[i].dim != grids[0].dim || grids[i].dtype != grids[0].dtype)
            return cfail(SGH_ERR_ARG, "all grids of a combination set need one dimension and one dtype");
    return SGH_OK;
}

int combi_build(sgh_combi *c) {
    const int d = c->d;
    std::vector<std::vector<int32_t>> order;
    int rc = subspaces_of(c->grids.data(), static_cast<int>(c->grids.size()), order);
    if (rc) return rc;
    auto norm = norm1;
    c->sub_levels.clear();
    c->sub_offsets.clear();
    int64_t off = 0;
    for (const auto &m : order) {
        c->sub_levels.insert(c->sub_levels.end(), m.begin(), m.end());
        c->sub_offsets.push_back(off);
        off += int64_t(1) << (norm(m) - d);
    }
    c->total = off;
    // contributors (grid list order) and gather units
    std::vector<int32_t> cbegin;
    std::vector<int32_t> &cgrid = c->cgrid;
    std::vector<double> ccoef;
    cgrid.clear();
    c->csub.clear();
    std::vector<CombiUnit> gunits;
    for (size_t s = 0; s < order.size(); ++s) {
        cbegin.push_back(static_cast<int32_t>(cgrid.size()));
        for (size_t g = 0; g < c->grids.size(); ++g) {
            bool in = true;
            for (int k = 0; k < d && in; ++k) in = order[s][static_cast<size_t>(k)] <= c->grids[g].level[k];
            if (in) {
                cgrid.push_back(static_cast<int32_t>(g));
                c->csub.push_back(static_cast<int32_t>(s));
                ccoef.push_back(c->coefs[g]);
            }
        }
        const int64_t size = int64_t(1) << (norm(order[s]) - d);
        for (int64_t st = 0; st < size; st += 256)
            gunits.push_back(CombiUnit{static_cast<int32_t>(s), static_cast<int32_t>(std::min<int64_t>(256, size - st)), st});
    }
    if (cgrid.size() > 0x7fffffff) return cfail(SGH_ERR_UNSUPPORTED, "too many (subspace, grid) pairs");
    cbegin.push_back(static_cast<int32_t>(cgrid.size()));
    // scatter: dense table level vector -> subspace offset
    int64_t tsize = 1;
    for (int k = 0; k < d; ++k) {
        int maxL = 1;
        for (const auto &g : c->grids) maxL = std::max(maxL, g.level[k]);
        c->tstride[k] = tsize;
        tsize *= maxL;
        if (tsize > kMaxTable) return cfail(SGH_ERR_UNSUPPORTED, "sparse-grid level table too large");
    }
    std::vector<int64_t> table(static_cast<size_t>(tsize), -1);
    for (size_t s = 0; s < order.size(); ++s) {
        int64_t t = 0;
        for (int k = 0; k < d; ++k) t += (order[s][static_cast<size_t>(k)] - 1) * c->tstride[k];
        table[static_cast<size_t>(t)] = c->sub_offsets[s];
    }
    std::vector<CombiUnit> sunits;
    for (size_t g = 0; g < c->grids.size(); ++g) {
        int64_t N = 1;
        for (int k = 0; k < d; ++k) N *= (int64_t(1) << c->grids[g].level[k]) - 1;
        for (int64_t st = 0; st < N; st += 256)
            sunits.push_back(CombiUnit{static_cast<int32_t>(g), static_cast<int32_t>(std::min<int64_t>(256, N - st)), st});
    }
    if (gunits.size() > 0x7fffffff || sunits.size() > 0x7fffffff) return cfail(SGH_ERR_UNSUPPORTED, "too many work units");
    c->ngunits = static_cast<int32_t>(gunits.size());
    c->nsunits = static_cast<int32_t>(sunits.size());
    hipError_t e = upload(&c->d_grids, grid_table(*c));
    if (e == hipSuccess) e = upload(&c->d_sub_levels, c->sub_levels);
    if (e == hipSuccess) e = upload(&c->d_sub_offsets, c->sub_offsets);
    if (e == hipSuccess) e = upload(&c->d_cbegin, cbegin);
    if (e == hipSuccess) e = upload_contrib(c);
    if (e == hipSuccess) e = upload(&c->d_ccoef, ccoef);
    if (e == hipSuccess) e = upload(&c->d_table, table);
    if (e == hipSuccess) e = upload(&c->d_gunits, gunits);
    if (e == hipSuccess) e = upload(&c->d_sunits, sunits);
    if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
    return SGH_OK;
}

void drop_graph(sgh_combi *c) {
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
    c->graph_sparse = nullptr;
}

// hierarchize all grids, gather, scatter, dehierarchize all grids
int reduce_launches(sgh_combi *c, void *sparse, hipStream_t s) {
    int rc = sgh_plan_execute(c->hier, s);
    if (rc) return rc;
    hipError_t e = do_gather(*c, sparse, s);
    if (e == hipSuccess) e = do_scatter(*c, sparse, s);
    if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
    return sgh_plan_execute(c->dehier, s);
}

}  // namespace
}  // namespace sgh

extern "C" {

int sgh_combi_create(sgh_combi **out, const sgh_grid *grids, int32_t n, const double *coefs, uint32_t flags) {
    using namespace sgh;
    if (!out) return cfail(SGH_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (!coefs) return cfail(SGH_ERR_ARG, "null coefficients");
    int rc = check_set(grids, n);
    if (rc) return rc;
    std::unique_ptr<sgh_combi, void (*)(sgh_combi *)> c(new (std::nothrow) sgh_combi, combi_free);
    if (!c) return cfail(SGH_ERR_NOMEM, "allocation");
    c->d = grids[0].dim;
    c->dtype = grids[0].dtype;
    c->flags = flags;
    c->grids.assign(grids, grids + n);
    c->coefs.assign(coefs, coefs + n);
    rc = combi_build(c.get());
    if (rc) return rc;
    rc = sgh_plan_create(&c->hier, SGH_OP_HIERARCHIZE, grids, n, flags & SGH_PLAN_AUTOTUNE);
    if (rc) return rc;
    rc = sgh_plan_create(&c->dehier, SGH_OP_DEHIERARCHIZE, grids, n, flags & SGH_PLAN_AUTOTUNE);
    if (rc) return rc;
    *out = c.release();
    return SGH_OK;
}

int64_t sgh_combi_sparse_points(const sgh_combi *c) { return c ? c->total : -1; }

int32_t sgh_combi_num_subspaces(const sgh_combi *c) {
    return c ? static_cast<int32_t>(c->sub_offsets.size()) : -1;
}

int sgh_combi_layout(const sgh_combi *c, int32_t *sub_levels, int64_t *offsets) {
    if (!c || !sub_levels || !offsets) return sgh::cfail(SGH_ERR_ARG, "null argument");
    std::memcpy(sub_levels, c->sub_levels.data(), c->sub_levels.size() * sizeof(int32_t));
    std::memcpy(offsets, c->sub_offsets.data(), c->sub_offsets.size() * sizeof(int64_t));
    return SGH_OK;
}

int sgh_combi_gather(sgh_combi *c, void *sparse, void *stream) {
    if (!c || !sparse) return sgh::cfail(SGH_ERR_ARG, "null argument");
    hipError_t e = sgh::do_gather(*c, sparse, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SGH_OK : sgh::cfail(SGH_ERR_HIP, hipGetErrorString(e));
}

int sgh_combi_scatter(sgh_combi *c, const void *sparse, void *stream) {
    if (!c || !sparse) return sgh::cfail(SGH_ERR_ARG, "null argument");
    hipError_t e = sgh::do_scatter(*c, sparse, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SGH_OK : sgh::cfail(SGH_ERR_HIP, hipGetErrorString(e));
}

int sgh_combi_reduce(sgh_combi *c, void *sparse, void *stream) {
    using namespace sgh;
    if (!c || !sparse) return cfail(SGH_ERR_ARG, "null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!(c->flags & SGH_PLAN_GRAPH)) return reduce_launches(c, sparse, st);
    if (!c->exec || c->graph_sparse != sparse) {
        drop_graph(c);
        if (!c->cap) {
            hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
            if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
        }
        hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
        const int rc = reduce_launches(c, sparse, c->cap);
        e = hipStreamEndCapture(c->cap, &c->graph);
        if (rc) return rc;
        if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
        e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
        c->graph_sparse = sparse;
    }
    hipError_t e = hipGraphLaunch(c->exec, st);
    return e == hipSuccess ? SGH_OK : cfail(SGH_ERR_HIP, hipGetErrorString(e));
}

int sgh_combi_set_data(sgh_combi *c, const sgh_grid *grids, int32_t n) {
    using namespace sgh;
    if (!c || !grids || n != static_cast<int32_t>(c->grids.size())) return cfail(SGH_ERR_ARG, "grid count mismatch");
    for (int i = 0; i < n; ++i) {
        bool same = grids[i].dim == c->d && grids[i].dtype == c->dtype;
        for (int k = 0; same && k < c->d; ++k) same = grids[i].level[k] == c->grids[static_cast<size_t>(i)].level[k];
        if (!same) return cfail(SGH_ERR_ARG, "grid shape or dtype differs from the set");
    }
    int rc = sgh_plan_set_data(c->hier, grids, n);  // validates and synchronizes the device
    if (rc) return rc;
    rc = sgh_plan_set_data(c->dehier, grids, n);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) c->grids[static_cast<size_t>(i)].data = grids[i].data;
    hipError_t e = upload(&c->d_grids, grid_table(*c));
    if (e == hipSuccess) e = upload_contrib(c);
    if (e != hipSuccess) return cfail(SGH_ERR_HIP, hipGetErrorString(e));
    drop_graph(c);
    return SGH_OK;
}

int sgh_sparse_layout(const sgh_grid *grids, int32_t n, int32_t capacity, int32_t *sub_levels, int64_t *offsets,
                      int32_t *num_subspaces, int64_t *points) {
    using namespace sgh;
    if (n < 1 || !grids) return cfail(SGH_ERR_ARG, "need at least one grid");
    // shapes only: give grids without data disjoint placeholder addresses
    std::vector<sgh_grid> g(grids, grids + n);
    uintptr_t fake = 256;
    for (auto &x : g) {
        if (x.data) continue;
        x.data = reinterpret_cast<void *>(fake);
        const int64_t np = sgh_num_points(&x);
        if (np < 0) break;  // reported by check_set below
        fake += static_cast<uintptr_t>(np) * 8 + 256;
    }
    int rc = check_set(g.data(), n);
    if (rc) return rc;
    std::vector<std::vector<int32_t>> order;
    rc = subspaces_of(g.data(), n, order);
    if (rc) return rc;
    const int d = grids[0].dim;
    int64_t off = 0;
    for (size_t s = 0; s < order.size(); ++s) {
        if (static_cast<int64_t>(s) < capacity) {
            if (sub_levels) std::memcpy(sub_levels + s * d, order[s].data(), sizeof(int32_t) * static_cast<size_t>(d));
            if (offsets) offsets[s] = off;
        }
        off += int64_t(1) << (norm1(order[s]) - d);
    }
    if (num_subspaces) *num_subspaces = static_cast<int32_t>(order.size());
    if (points) *points = off;
    return SGH_OK;
}

void sgh_combi_destroy(sgh_combi *c) {
    if (c) sgh::combi_free(c);
}

}  // extern "C"
