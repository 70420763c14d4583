// Host side of the hierarchization library: descriptor validation, the
// per-grid launch schedule, batched plans with HIP-graph capture, the
// autotuner and event timing.  The C ABI is declared in include/sgh.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "sgh.h"
#include "sgh_internal.h"

namespace sgh {
namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(SGH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t esize_of(int dtype) { return dtype == SGH_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// Validation (all or nothing).
// relative: data holds a byte offset into a buffer given later (0 allowed).
int validate_one(const sgh_grid &g, int idx, int64_t *npoints, bool relative = false) {
    if (g.dim < 1 || g.dim > SGH_MAX_DIM) return fail(SGH_ERR_ARG, "grid %d: dim %d outside 1..%d", idx, g.dim, SGH_MAX_DIM);
    if (g.dtype != SGH_F32 && g.dtype != SGH_F64) return fail(SGH_ERR_DTYPE, "grid %d: dtype %d", idx, g.dtype);
    // the product of 2^l_k - 1 must fit in int64 together with the element size
    double log2n = 0.0;
    int64_t n = 1;
    for (int k = 0; k < g.dim; ++k) {
        const int L = g.level[k];
        if (L < 1 || L > SGH_MAX_LEVEL) return fail(SGH_ERR_ARG, "grid %d: level[%d] = %d outside 1..%d", idx, k, L, SGH_MAX_LEVEL);
        log2n += L;
    }
    if (log2n > 58.0) return fail(SGH_ERR_ARG, "grid %d: too many points (|l|_1 = %.0f)", idx, log2n);
    for (int k = 0; k < g.dim; ++k) n *= (int64_t(1) << g.level[k]) - 1;
    if (g.data == nullptr && !relative) return fail(SGH_ERR_ARG, "grid %d: null data pointer", idx);
    if (reinterpret_cast<uintptr_t>(g.data) % esize_of(g.dtype) != 0)
        return fail(SGH_ERR_ALIGN, "grid %d: data %p not aligned to %zu bytes", idx, g.data, esize_of(g.dtype));
    *npoints = n;
    return SGH_OK;
}

int validate_all(const sgh_grid *grids, int32_t n, bool relative = false) {
    if (n < 0) return fail(SGH_ERR_ARG, "negative grid count %d", n);
    if (n > 0 && grids == nullptr) return fail(SGH_ERR_ARG, "null grid array");
    std::vector<std::pair<uintptr_t, uintptr_t>> spans;
    spans.reserve(n);
    for (int i = 0; i < n; ++i) {
        int64_t np = 0;
        int rc = validate_one(grids[i], i, &np, relative);
        if (rc) return rc;
        const uintptr_t b = reinterpret_cast<uintptr_t>(grids[i].data);
        spans.emplace_back(b, b + static_cast<uintptr_t>(np) * esize_of(grids[i].dtype));
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second)
            return fail(SGH_ERR_OVERLAP, "grids overlap in memory at %p", reinterpret_cast<void *>(spans[i].first));
    return SGH_OK;
}

// ---------------------------------------------------------------------------
// Geometry: level-1 axes (a single point) are the identity and leave the
// strides of the other axes unchanged, so they are dropped.
struct Geom {
    int d = 0;
    int L[kMaxDim] = {};
    int64_t n[kMaxDim] = {};
    int64_t st[kMaxDim] = {};
    int64_t N = 1;
    int dtype = SGH_F64;
    void *data = nullptr;
};

Geom make_geom(const sgh_grid &g) {
    Geom r;
    r.dtype = g.dtype;
    r.data = g.data;
    int64_t st = 1;
    for (int k = 0; k < g.dim; ++k) {
        const int L = g.level[k];
        const int64_t nk = (int64_t(1) << L) - 1;
        if (L >= 2) {
            r.L[r.d] = L;
            r.n[r.d] = nk;
            r.st[r.d] = st;
            ++r.d;
        }
        st *= nk;
    }
    r.N = st;
    return r;
}

TileGeom make_tile_geom(const Geom &g, int m) {
    TileGeom t{};
    t.m = m;
    for (int k = 0; k < m; ++k) {
        t.L[k] = g.L[k];
        t.n[k] = static_cast<int32_t>(g.n[k]);
        t.st[k] = static_cast<int32_t>(g.st[k]);
        t.rst[k] = 1.0f / static_cast<float>(g.st[k]);
        t.rn[k] = 1.0f / static_cast<float>(g.n[k]);
    }
    return t;
}

// ---------------------------------------------------------------------------
// Device properties.
struct DevInfo {
    int cus = 256;
    int lds_per_cu = 160 * 1024;
    int max_lds_block = 160 * 1024;
    std::string arch = "gfx950";
};

DevInfo &dev_info() {
    static std::mutex mu;
    static std::map<int, DevInfo> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    DevInfo di;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        di.cus = prop.multiProcessorCount;
        if (prop.maxSharedMemoryPerMultiProcessor > 0) di.lds_per_cu = static_cast<int>(prop.maxSharedMemoryPerMultiProcessor);
        if (prop.sharedMemPerBlock > 0) di.max_lds_block = static_cast<int>(prop.sharedMemPerBlock);
        di.arch = prop.gcnArchName;
        const size_t colon = di.arch.find(':');
        if (colon != std::string::npos) di.arch = di.arch.substr(0, colon);
    }
    return cache.emplace(dev, di).first->second;
}

// ---------------------------------------------------------------------------
// Tuning cache: key -> "v1 v2 ..." (integers).  Filled by the autotuner,
// persisted to $SGH_AUTOTUNE_CACHE when set.
std::mutex g_tune_mu;
std::map<std::string, std::vector<int>> g_tune;
bool g_tune_loaded = false;

const char *tune_path() { return std::getenv("SGH_AUTOTUNE_CACHE"); }

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *p = tune_path();
    if (!p) return;
    std::ifstream in(p);
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ss(line);
        std::string key;
        if (!(ss >> key)) continue;
        std::vector<int> v;
        int x;
        while (ss >> x) v.push_back(x);
        if (!v.empty()) g_tune[key] = v;
    }
}

bool tune_get(const std::string &key, std::vector<int> *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_put(const std::string &key, const std::vector<int> &v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = v;
    const char *p = tune_path();
    if (!p) return;
    std::ofstream out(p, std::ios::trunc);
    out << "# sgh autotune cache v1\n";
    for (auto &kv : g_tune) {
        out << kv.first;
        for (int x : kv.second) out << ' ' << x;
        out << '\n';
    }
}

// ---------------------------------------------------------------------------
// Timing.
struct TimedLaunch {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_time_mu;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;
std::map<std::string, std::pair<int64_t, double>> g_time_acc;

bool timing_on(hipStream_t s) {
    if (!g_timing) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone) return false;
    return true;
}

struct TimerScope {
    bool on = false;
    hipEvent_t a{}, b{};
    hipStream_t s{};
    std::string name;
    TimerScope(const std::string &nm, hipStream_t st) : s(st), name(nm) {
        on = timing_on(st);
        if (!on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            on = false;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    ~TimerScope() {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_time_mu);
        g_timed.push_back({name, a, b});
    }
};

void timing_drain_locked() {
    for (auto &t : g_timed) {
        float ms = 0.f;
        if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            auto &acc = g_time_acc[t.name];
            acc.first += 1;
            acc.second += ms;
        }
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    g_timed.clear();
}

// ---------------------------------------------------------------------------
// Schedule of one grid: a list of launches, applied in order.
struct Step {
    enum Kind { TILE, POLE, TW, SPLIT, BOX } kind = TILE;
    TileLaunch tile{};
    TileTune ttune{};
    PoleLaunch pole{};
    PoleTune ptune{};
    TWLaunch tw{};
    SplitLaunch split{};
    BoxLaunch box{};
    std::vector<int> axes;  // axes (of the reduced geometry) this launch transforms
    int key = 0;            // largest axis covered; orders the inverse/transpose schedule
};

// Per-level override of the pole block exponent (0 = default), set through
// sgh_set_pole_block, and the fusion switch set through sgh_set_fusion.
std::mutex g_override_mu;
int g_pole_B_override[SGH_MAX_LEVEL + 1] = {};
int g_pole3_override[SGH_MAX_LEVEL + 1] = {};  // 1 + TB * 100 + B * 10 + pf, 0 = none
int g_fusion = 1;
int g_walk_pref = 0;  // 0: smallest-stride walk candidate, 1: largest
int g_split_fine = 0;    // block span exponent of the first split phase, 0 = largest that fits
int g_box_bytes = 0;     // largest box launch tile in bytes, 0 = default
int g_box_row = 0;       // smallest box row (columns * element size) in bytes, 0 = default
int g_split_coarse = 0;  // the same for the later phases, 0 = default
int g_outer_stencil = 1; // hierarchization: fold the axis after a three-level walk into the fused launch
int g_tw_xcd = 0;        // fused launches: consecutive pencils on one XCD

int pole_B_override(int L) {
    std::lock_guard<std::mutex> lk(g_override_mu);
    return (L >= 0 && L <= SGH_MAX_LEVEL) ? g_pole_B_override[L] : 0;
}

int pole3_override(int L) {
    std::lock_guard<std::mutex> lk(g_override_mu);
    return (L >= 0 && L <= SGH_MAX_LEVEL) ? g_pole3_override[L] : 0;
}

int fusion_level() {
    std::lock_guard<std::mutex> lk(g_override_mu);
    return g_fusion;
}

int default_pole_B(int L) {
    const int o = pole_B_override(L);
    if (o > 0) return o;
    switch (L) {
        case 7: return 4;
        case 8: return 4;
        case 9: return 5;
        case 10: return 5;
        default: return L;
    }
}

// Block exponent of a walked axis in the fused kernel (small register state).
int default_tw_B(int L) {
    switch (L) {
        case 2: return 2;
        case 3: return 3;
        case 4: return 2;
        case 5: return 3;
        case 6: return 3;
        case 7: return 4;
        case 8: return 4;
        default: return 0;
    }
}

int pow2_ceil(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Largest number of elements a tile may hold in LDS for this element size.
int64_t tile_capacity(int dtype) { return dtype == SGH_F64 ? 8192 : 16384; }

void choose_tile_tune(int64_t chunk, TileTune *t) {
    int nt = 256;
    if (chunk > 256 * 32) nt = 512;
    int ept = pow2_ceil(static_cast<int>((chunk + nt - 1) / nt));
    if (ept < 1) ept = 1;
    t->nt = nt;
    t->ept = ept;
    t->grid = 0;
}

std::string grid_key(int op, const Geom &g) {
    std::ostringstream ss;
    ss << dev_info().arch << ":op" << op << ":dt" << g.dtype << ":l";
    for (int k = 0; k < g.d; ++k) ss << (k ? "," : "") << g.L[k];
    return ss.str();
}

// Choices a schedule is built from.  walk: -1 = default, -2 = no fused walk,
// k >= 0 = walk axis k.  tile_mult: tiles per LDS chunk (0 = default).
// pole_code[k]: B * 1000 + workgroup size for strided axis k (0 = default).
struct SchedOpts {
    int walk = -1;
    bool walk_two_level = false;  // force the two-level walk in the fused kernel
    int outer = -1;               // fold the next axis into a three-level walk: -1 knob, 0 no, 1 yes
    bool oop = false;             // out-of-place schedule (its first launch reads the source grid)
    int tile_mult = 0;
    std::vector<int> pole_code;
};

// Pole codes: two-level  B * 1000 + nt;  three-level  1000000 + TB * 100000 +
// pf * 10000 + B * 1000 + nt.
int pole_code2(int B, int nt) { return B * 1000 + nt; }
int pole_code3(int TB, int B, int pf, int nt) { return 1000000 + TB * 100000 + pf * 10000 + B * 1000 + nt; }

// Default three-level split of a strided pole (0 = keep the two-level walk).
bool default_pole3(int L, int *TB, int *B) {
    switch (L) {
        case 8: *TB = 2; *B = 3; return true;
        case 9: *TB = 3; *B = 3; return true;
        case 10: *TB = 2; *B = 4; return true;
        default: return false;
    }
}

// Tuning-cache layout per grid: [tile_mult, pole_code_1 .. pole_code_{d-1}, walk code]
// with walk code 0 = default, 1 = none, 2 + k = axis k, 100 + k = axis k with
// the two-level walk.
SchedOpts opts_from_tuned(const Geom &g, const std::vector<int> &t) {
    SchedOpts o;
    o.pole_code.assign(static_cast<size_t>(g.d), 0);
    if (!t.empty()) o.tile_mult = t[0];
    for (int k = 1; k < g.d && static_cast<size_t>(k) < t.size(); ++k) o.pole_code[static_cast<size_t>(k)] = t[static_cast<size_t>(k)];
    if (t.size() > static_cast<size_t>(g.d)) {
        const int w = t[static_cast<size_t>(g.d)];
        if (w >= 100) {
            o.walk = w - 100;
            o.walk_two_level = true;
        } else {
            o.walk = w == 0 ? -1 : (w == 1 ? -2 : w - 2);
        }
    }
    return o;
}

std::vector<int> tuned_from_opts(const Geom &g, const SchedOpts &o) {
    std::vector<int> t(static_cast<size_t>(g.d) + 1, 0);
    t[0] = o.tile_mult;
    for (int k = 1; k < g.d; ++k)
        t[static_cast<size_t>(k)] = static_cast<size_t>(k) < o.pole_code.size() ? o.pole_code[static_cast<size_t>(k)] : 0;
    t[static_cast<size_t>(g.d)] =
        o.walk == -1 ? 0 : (o.walk == -2 ? 1 : (o.walk_two_level ? 100 + o.walk : o.walk + 2));
    return t;
}

// Number of leading axes that fit one LDS tile, and the tile size.
int tile_axes(const Geom &g, int64_t *Sm_out) {
    const int64_t cap = tile_capacity(g.dtype);
    int m = 0;
    int64_t Sm = 1;
    while (m < g.d && Sm * g.n[m] <= cap) {
        Sm *= g.n[m];
        ++m;
    }
    *Sm_out = Sm;
    return m;
}

// Can axis w (>= m) be walked by the fused kernel over a tile of Sm points?
bool walk_ok(const Geom &g, int m, int64_t Sm, int w) {
    if (m < 1 || w < m || w >= g.d || Sm > 4 * kTWThreads) return false;
    const int L = g.L[w];
    const int ept = Sm <= kTWThreads ? 1 : (Sm <= 2 * kTWThreads ? 2 : 4);
    const bool three = ept == 1 && tw3_supported(L, L - 6, 3) && fusion_level() != 2;
    if (!tw_supported(L, default_tw_B(L), ept) && !three) return false;
    // the pencil's byte offsets must fit the 32-bit buffer window
    const int64_t bytes = g.n[w] * g.st[w] * static_cast<int64_t>(esize_of(g.dtype));
    return bytes < (int64_t(1) << 32) - 1;
}

// Walk candidates of a grid (largest stride first).
std::vector<int> walk_candidates(const Geom &g) {
    std::vector<int> c;
    int64_t Sm = 1;
    const int m = tile_axes(g, &Sm);
    if (m >= g.d) return c;
    for (int w = g.d - 1; w >= m; --w)
        if (walk_ok(g, m, Sm, w)) c.push_back(w);
    return c;
}

// Columns per box-launch workgroup for a group of P points: the widest of
// 64, 32, 16 adjacent columns whose box fits `bytes` with rows of at least
// `row` bytes, or 0.
struct BoxLimits {
    int64_t bytes = 65536;
    int row = 128;
};

BoxLimits box_limits() {
    std::lock_guard<std::mutex> lk(g_override_mu);
    BoxLimits b;
    if (g_box_bytes > 0) b.bytes = g_box_bytes;
    if (g_box_row > 0) b.row = g_box_row;
    return b;
}

// Largest box the box kernel is built for: 512 threads of at most 32 elements.
constexpr int64_t kBoxMaxElems = 512 * 32;

int box_width(int64_t P, int esize, const BoxLimits &lim) {
    for (int W : {64, 32, 16})
        if (P * W * esize <= lim.bytes && P * W <= kBoxMaxElems && W * esize >= lim.row) return W;
    return 0;
}

// Launches of the dyadic split of axis k: phases with lattice exponents
// E = 0, B0, B0 + B1, ... until the whole remaining pole fits one block;
// fine to coarse for the hierarchization, coarse to fine otherwise.
void split_steps(int op, const Geom &g, int k, std::vector<Step> *steps) {
    const int64_t S = g.st[k];
    int W = 1;
    while (W < 64 && W < S) W <<= 1;
    const int esize = g.dtype == SGH_F64 ? 8 : 4;
    const int bmax = split_max_span(W, esize);
    // 32 KiB tiles: four or five workgroups per CU keep enough loads in flight
    int fine = std::max(1, bmax - 1), coarse = std::min(bmax, 7);
    {
        std::lock_guard<std::mutex> lk(g_override_mu);
        if (g_split_fine > 0) fine = std::min(bmax, g_split_fine);
        if (g_split_coarse > 0) coarse = std::min(bmax, g_split_coarse);
    }
    std::vector<Step> phases;
    for (int E = 0; E < g.L[k];) {
        Step s;
        s.kind = Step::SPLIT;
        s.axes = {k};
        s.key = k;
        s.split.data = g.data;
        s.split.S = S;
        s.split.outer = g.N / (g.n[k] * S);
        s.split.L = g.L[k];
        s.split.E = E;
        // the coarse phases work on few points: narrow blocks spread them over
        // many workgroups
        s.split.Bs = std::min(E == 0 ? fine : coarse, g.L[k] - E);
        s.split.W = W;
        E += s.split.Bs;
        // a lattice of one point (the root) changes only under the transpose
        if (op == SGH_OP_ADJOINT || g.L[k] - s.split.E > 1) phases.push_back(s);
    }
    if (op != SGH_OP_HIERARCHIZE) std::reverse(phases.begin(), phases.end());
    steps->insert(steps->end(), phases.begin(), phases.end());
}

std::vector<Step> build_schedule_opts(int op, const Geom &g, const SchedOpts &o) {
    std::vector<Step> steps;
    if (g.d == 0) return steps;
    const int64_t cap = tile_capacity(g.dtype);
    int64_t Sm = 1;
    int m = tile_axes(g, &Sm);
    int walk = -1, folded = -1;
    if (m >= 1 && m < g.d && fusion_level() >= 1 && o.walk != -2) {
        if (o.walk >= 0 && walk_ok(g, m, Sm, o.walk)) {
            walk = o.walk;
        } else if (o.walk == -1) {
            // default: the walk candidate with the smallest stride, so that a
            // pencil is one contiguous slab of the grid
            auto c = walk_candidates(g);
            int pref = 0;
            {
                std::lock_guard<std::mutex> lk(g_override_mu);
                pref = g_walk_pref;
            }
            if (!c.empty()) walk = pref == 1 ? c.front() : c.back();
        }
    }
    if (walk >= 0) {
        Step s;
        s.kind = Step::TW;
        for (int k = 0; k < m; ++k) s.axes.push_back(k);
        s.axes.push_back(walk);
        s.key = walk;
        s.tw.data = g.data;
        s.tw.Sm = static_cast<int32_t>(Sm);
        s.tw.Sw = g.st[walk];
        s.tw.mid = g.st[walk] / Sm;
        s.tw.nwg = (g.N / (g.n[walk] * g.st[walk])) * s.tw.mid;
        s.tw.L = g.L[walk];
        s.tw.B = default_tw_B(g.L[walk]);
        s.tw.ept = Sm <= kTWThreads ? 1 : (Sm <= 2 * kTWThreads ? 2 : 4);
        const bool two_ok = tw_supported(s.tw.L, s.tw.B, s.tw.ept);
        const bool three_ok = s.tw.ept == 1 && tw3_supported(s.tw.L, s.tw.L - 6, 3) && fusion_level() != 2;
        if (three_ok && !(o.walk_two_level && two_ok)) {
            s.tw.split = 3;
            s.tw.TB = s.tw.L - 6;
            s.tw.B = 3;
        }
        s.tw.g = make_tile_geom(g, m);
        int outer = 0;
        {
            std::lock_guard<std::mutex> lk(g_override_mu);
            outer = o.outer >= 0 ? o.outer : g_outer_stencil;
            s.tw.xcd = g_tw_xcd;
        }
        if (o.oop && op == SGH_OP_HIERARCHIZE && s.tw.split == 3 && outer && walk + 1 < g.d) {
            // the next axis's one-shot stencil is applied as the pencil's rows are
            // read (out of place only: the predecessor planes are read while
            // other workgroups transform them)
            s.tw.oL = g.L[walk + 1];
            s.tw.on = static_cast<int32_t>(g.n[walk + 1]);
            s.axes.push_back(walk + 1);
            s.key = walk + 1;
            folded = walk + 1;
        }
        steps.push_back(s);
    } else if (m >= 1) {
        Step s;
        s.kind = Step::TILE;
        for (int k = 0; k < m; ++k) s.axes.push_back(k);
        s.key = m - 1;
        s.tile.data = g.data;
        s.tile.total = g.N;
        s.tile.g = make_tile_geom(g, m);
        int64_t target = std::max<int64_t>(Sm, std::min<int64_t>(cap, 2048));
        if (o.tile_mult > 0) target = std::min<int64_t>(cap, Sm * o.tile_mult);
        int64_t mult = std::max<int64_t>(1, target / Sm);
        if (m == g.d) mult = 1;  // the whole grid is one tile
        s.tile.chunk = static_cast<int32_t>(Sm * mult);
        choose_tile_tune(s.tile.chunk, &s.ttune);
        steps.push_back(s);
    } else {
        // axis 0 too long for a tile: dyadic block split
        split_steps(op, g, 0, &steps);
        m = 1;
    }
    for (int k = m; k < g.d; ++k) {
        if (k == walk || k == folded) continue;
        if (fusion_level() >= 1) {
            // consecutive small strided axes: one box launch for all of them
            const BoxLimits lim = box_limits();
            const int es = g.dtype == SGH_F64 ? 8 : 4;
            int kend = k, W = box_width(g.n[k], es, lim);
            int64_t P = g.n[k];
            while (kend + 1 < g.d && kend + 1 != walk && kend + 1 != folded &&
                   box_width(P * g.n[kend + 1], es, lim) > 0) {
                P *= g.n[++kend];
                W = box_width(P, es, lim);
            }
            if (kend > k) {
                Step s;
                s.kind = Step::BOX;
                for (int a = k; a <= kend; ++a) s.axes.push_back(a);
                s.key = kend;
                s.box.data = g.data;
                s.box.S = g.st[k];
                s.box.P = static_cast<int32_t>(P);
                s.box.W = W;
                s.box.outer = g.N / (g.st[k] * P);
                TileGeom &tg = s.box.g;
                tg.m = kend - k + 1;
                int64_t st = W;
                for (int a = 0; a < tg.m; ++a) {
                    tg.L[a] = g.L[k + a];
                    tg.n[a] = static_cast<int32_t>(g.n[k + a]);
                    tg.st[a] = static_cast<int32_t>(st);
                    tg.rst[a] = 1.0f / static_cast<float>(st);
                    tg.rn[a] = 1.0f / static_cast<float>(g.n[k + a]);
                    st *= g.n[k + a];
                }
                choose_tile_tune(P * W, &s.ttune);
                if (s.ttune.ept < 4) s.ttune.ept = 4;
                steps.push_back(s);
                k = kend;
                continue;
            }
        }
        const int L = g.L[k];
        int B = default_pole_B(L);
        int nt = 256;
        int split = 2, TB = 0, pf = 0;
        const int o3 = pole3_override(L);
        if (o3 > 0) {
            split = 3;
            TB = (o3 - 1) / 100;
            B = ((o3 - 1) / 10) % 10;
            pf = (o3 - 1) % 10;
        } else if (pole_B_override(L) == 0) {
            int tb3 = 0, b3 = 0;
            if (default_pole3(L, &tb3, &b3)) {
                split = 3;
                TB = tb3;
                B = b3;
                pf = 1;
            }
        }
        const int code = static_cast<size_t>(k) < o.pole_code.size() ? o.pole_code[static_cast<size_t>(k)] : 0;
        if (o3 > 0) {
            // forced split; ignore the tuned choice
        } else if (pole_B_override(L) == 0 && code >= 1000000) {
            const int c = code - 1000000;
            const int tb = c / 100000, cpf = (c / 10000) % 10, cb = (c / 1000) % 10, cnt = c % 1000;
            if (pole3_supported(L, tb, cb) && cnt == 256) {
                split = 3;
                TB = tb;
                B = cb;
                pf = cpf;
                nt = cnt;
            }
        } else if (pole_B_override(L) == 0 && code > 0 && pole_supported(L, code / 1000)) {
            split = 2;
            B = code / 1000;
            nt = code % 1000;
            if (nt != 64 && nt != 128 && nt != 256 && nt != 512) nt = 256;
        }
        if (L <= kPoleMaxLevel && (split == 3 ? pole3_supported(L, TB, B) : pole_supported(L, B))) {
            Step s;
            s.kind = Step::POLE;
            s.axes = {k};
            s.key = k;
            s.pole.data = g.data;
            s.pole.npoles = g.N / g.n[k];
            s.pole.S = g.st[k];
            s.pole.L = L;
            s.pole.B = B;
            s.pole.split = split;
            s.pole.TB = TB;
            s.pole.pf = pf;
            s.ptune.nt = nt;
            steps.push_back(s);
        } else {
            split_steps(op, g, k, &steps);
        }
    }
    if (op != SGH_OP_HIERARCHIZE) {
        // Inverse and transpose: launches in reverse axis order; the split
        // phases of one long pole keep their coarse-to-fine order.
        std::stable_sort(steps.begin(), steps.end(), [](const Step &a, const Step &b) { return a.key > b.key; });
    }
    return steps;
}

// The schedule the library uses: autotuned choices when cached, else defaults.
std::vector<Step> build_schedule(int op, const Geom &g, bool oop = false) {
    std::vector<int> tuned;
    SchedOpts o;
    if (tune_get(grid_key(op, g), &tuned)) o = opts_from_tuned(g, tuned);
    o.oop = oop;
    return build_schedule_opts(op, g, o);
}

void retarget_one(Step &s, void *data) {
    s.tile.data = data;
    s.pole.data = data;
    s.tw.data = data;
    s.split.data = data;
    s.box.data = data;
}

void retarget(std::vector<Step> &steps, void *data) {
    for (auto &s : steps) retarget_one(s, data);
}

const char *step_name(const Step &s) {
    switch (s.kind) {
        case Step::TILE: return "tile";
        case Step::POLE: return "pole";
        case Step::TW: return "tw";
        case Step::SPLIT: return "split";
        default: return "box";
    }
}

std::string step_timer_name(int op, int dtype, const Step &s) {
    std::ostringstream ss;
    static const char *ops[] = {"hier", "dehier", "adjoint"};
    ss << ops[op] << "_" << (dtype == SGH_F64 ? "f64" : "f32") << "_" << step_name(s);
    if (s.kind == Step::POLE) ss << "_L" << s.pole.L;
    if (s.kind == Step::TILE) ss << "_m" << s.tile.g.m;
    if (s.kind == Step::TW) {
        ss << "_m" << s.tw.g.m << "_L" << s.tw.L;
        if (s.tw.oL) ss << "_o" << s.tw.oL;
    }
    if (s.kind == Step::SPLIT) ss << "_L" << s.split.L << "_E" << s.split.E;
    if (s.kind == Step::BOX) ss << "_m" << s.box.g.m;
    return ss.str();
}

// Launch preconditions of one step (a kernel instantiation exists for it),
// checked for every step of a grid before the first of them is launched, so
// that a grid is never left partly transformed.
bool step_launchable(const Step &s) {
    switch (s.kind) {
        case Step::TILE:
            return tile_ept_supported(s.ttune.ept) && (s.ttune.nt == 128 || s.ttune.nt == 256 || s.ttune.nt == 512) &&
                   static_cast<int64_t>(s.ttune.nt) * s.ttune.ept >= s.tile.chunk;
        case Step::BOX:
            return (s.ttune.ept == 4 || s.ttune.ept == 8 || s.ttune.ept == 16 || s.ttune.ept == 32) &&
                   (s.ttune.nt == 256 || s.ttune.nt == 512) &&
                   static_cast<int64_t>(s.box.P) * s.box.W <= static_cast<int64_t>(s.ttune.nt) * s.ttune.ept;
        case Step::POLE:
            return s.pole.split == 3 ? pole3_supported(s.pole.L, s.pole.TB, s.pole.B) && s.ptune.nt == 256
                                     : pole_supported(s.pole.L, s.pole.B);
        case Step::TW:
            if (s.tw.oL > 0 && s.tw.split != 3) return false;
            return s.tw.split == 3 ? s.tw.ept == 1 && tw3_supported(s.tw.L, s.tw.TB, s.tw.B)
                                   : tw_supported(s.tw.L, s.tw.B, s.tw.ept);
        case Step::SPLIT:
            return s.split.W >= 1 && s.split.W <= 64 && s.split.Bs >= 1 && s.split.Bs <= s.split.L - s.split.E;
        default:
            return false;
    }
}

hipError_t run_step(int op, int dtype, const Step &s, hipStream_t st) {
    if (!step_launchable(s)) return hipErrorInvalidValue;
    TimerScope ts(step_timer_name(op, dtype, s), st);
    switch (s.kind) {
        case Step::TILE: return launch_tile(op, dtype, s.tile, s.ttune, st);
        case Step::POLE: return launch_pole(op, dtype, s.pole, s.ptune, st);
        case Step::TW: return launch_tw(op, dtype, s.tw, st);
        case Step::SPLIT: return launch_split(op, dtype, s.split, st);
        case Step::BOX: return launch_box(op, dtype, s.box, s.ttune, st);
        default: return hipErrorInvalidValue;
    }
}

// A schedule run out of place: the first launch reads src and writes dst
// (pole and fused launches take a destination), every later one works on dst
// in place; a schedule that starts with another kind of launch copies src to
// dst first.
hipError_t run_schedule_out(int op, int dtype, const std::vector<Step> &steps, void *src, void *dst, size_t bytes,
                            hipStream_t st) {
    size_t i0 = 0;
    if (!steps.empty() && (steps[0].kind == Step::TW || steps[0].kind == Step::POLE)) {
        Step f = steps[0];
        retarget_one(f, src);
        f.tw.dst = dst;
        f.pole.dst = dst;
        hipError_t e = run_step(op, dtype, f, st);
        if (e != hipSuccess) return e;
        i0 = 1;
    } else if (bytes) {
        hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    for (size_t i = i0; i < steps.size(); ++i) {
        Step s = steps[i];
        retarget_one(s, dst);
        s.tw.dst = nullptr;
        s.pole.dst = nullptr;
        hipError_t e = run_step(op, dtype, s, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

std::string describe_steps(int op, const Geom &g, const std::vector<Step> &steps) {
    std::ostringstream ss;
    ss << "{\"op\":" << op << ",\"dtype\":" << g.dtype << ",\"points\":" << g.N << ",\"launches\":[";
    int trips = 0;
    for (size_t i = 0; i < steps.size(); ++i) {
        const Step &s = steps[i];
        if (i) ss << ",";
        ss << "{\"kind\":\"" << step_name(s) << "\",\"axes\":[";
        for (size_t a = 0; a < s.axes.size(); ++a) ss << (a ? "," : "") << s.axes[a];
        ss << "]";
        if (s.kind == Step::TILE)
            ss << ",\"chunk\":" << s.tile.chunk << ",\"nt\":" << s.ttune.nt << ",\"ept\":" << s.ttune.ept;
        if (s.kind == Step::POLE)
            ss << ",\"L\":" << s.pole.L << ",\"B\":" << s.pole.B << ",\"split\":" << s.pole.split << ",\"TB\":" << s.pole.TB
               << ",\"prefetch\":" << s.pole.pf << ",\"nt\":" << s.ptune.nt;
        if (s.kind == Step::SPLIT)
            ss << ",\"L\":" << s.split.L << ",\"E\":" << s.split.E << ",\"Bs\":" << s.split.Bs << ",\"W\":" << s.split.W;
        if (s.kind == Step::BOX)
            ss << ",\"W\":" << s.box.W << ",\"box\":" << s.box.P * s.box.W << ",\"nt\":" << s.ttune.nt
               << ",\"ept\":" << s.ttune.ept;
        if (s.kind == Step::TW)
            ss << ",\"L\":" << s.tw.L << ",\"B\":" << s.tw.B << ",\"split\":" << s.tw.split << ",\"TB\":" << s.tw.TB
               << ",\"ept\":" << s.tw.ept << ",\"tile\":" << s.tw.Sm << ",\"workgroups\":" << s.tw.nwg
               << ",\"outer_level\":" << s.tw.oL << ",\"xcd_order\":" << s.tw.xcd;
        ss << "}";
        // the coarse split phases touch a small part of the grid
        trips += (s.kind == Step::SPLIT && s.split.E > 0) ? 0 : 1;
    }
    ss << "],\"hbm_round_trips\":" << trips << "}";
    return ss.str();
}

int copy_out(const std::string &s, char *buf, int32_t len) {
    if (buf && len > 0) {
        const size_t n = std::min<size_t>(s.size(), static_cast<size_t>(len - 1));
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return static_cast<int>(s.size()) + 1;
}

// ---------------------------------------------------------------------------
// One-shot transforms: every grid gets its own schedule.
int transform(int op, const sgh_grid *grids, int32_t n, void *stream) {
    if (op < 0 || op > 2) return fail(SGH_ERR_ARG, "unknown op %d", op);
    int rc = validate_all(grids, n);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<std::vector<Step>> all(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        all[static_cast<size_t>(i)] = build_schedule(op, make_geom(grids[i]));
        for (auto &s : all[static_cast<size_t>(i)])
            if (!step_launchable(s))
                return fail(SGH_ERR_UNSUPPORTED, "grid %d: no %s kernel for this shape under the current tuning knobs", i,
                            step_name(s));
    }
    for (int i = 0; i < n; ++i) {
        const int dtype = grids[i].dtype;
        for (auto &s : all[static_cast<size_t>(i)]) {
            hipError_t e = run_step(op, dtype, s, st);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
        }
    }
    return SGH_OK;
}

// Out of place: grid i of dst receives the transform of grid i of src (same
// shape and dtype); dst grids overlap no src grid and no other dst grid,
// except that dst[i] may be src[i] itself (then in place).
int transform_out(int op, const sgh_grid *src, const sgh_grid *dst, int32_t n, void *stream) {
    if (op < 0 || op > 2) return fail(SGH_ERR_ARG, "unknown op %d", op);
    int rc = validate_all(src, n);
    if (rc) return rc;
    rc = validate_all(dst, n);
    if (rc) return rc;
    std::vector<std::pair<uintptr_t, uintptr_t>> sspan, dspan;
    for (int i = 0; i < n; ++i) {
        const sgh_grid &a = src[i], &b = dst[i];
        bool same = a.dim == b.dim && a.dtype == b.dtype;
        for (int k = 0; same && k < a.dim; ++k) same = a.level[k] == b.level[k];
        if (!same) return fail(SGH_ERR_ARG, "grid %d: source and destination differ in shape or dtype", i);
        const uintptr_t bytes = static_cast<uintptr_t>(make_geom(a).N) * esize_of(a.dtype);
        sspan.emplace_back(reinterpret_cast<uintptr_t>(a.data), reinterpret_cast<uintptr_t>(a.data) + bytes);
        dspan.emplace_back(reinterpret_cast<uintptr_t>(b.data), reinterpret_cast<uintptr_t>(b.data) + bytes);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i == j && dspan[i].first == sspan[j].first) continue;  // in place
            if (dspan[i].first < sspan[j].second && sspan[j].first < dspan[i].second)
                return fail(SGH_ERR_OVERLAP, "destination %d overlaps source %d", i, j);
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<std::vector<Step>> all(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) {
        const bool inplace = dspan[i].first == sspan[i].first;
        all[static_cast<size_t>(i)] = build_schedule(op, make_geom(src[i]), !inplace);
        for (auto &s : all[static_cast<size_t>(i)])
            if (!step_launchable(s))
                return fail(SGH_ERR_UNSUPPORTED, "grid %d: no %s kernel for this shape under the current tuning knobs", i,
                            step_name(s));
    }
    for (int i = 0; i < n; ++i) {
        hipError_t e;
        if (dspan[i].first == sspan[i].first) {
            e = hipSuccess;
            for (auto &s : all[static_cast<size_t>(i)]) {
                e = run_step(op, src[i].dtype, s, st);
                if (e != hipSuccess) break;
            }
        } else {
            e = run_schedule_out(op, src[i].dtype, all[static_cast<size_t>(i)], src[i].data, dst[i].data,
                                 dspan[i].second - dspan[i].first, st);
        }
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
    }
    return SGH_OK;
}

// ---------------------------------------------------------------------------
// Batched plans.
struct BatchGroup {
    int dtype = SGH_F64;
    std::vector<int> grid_idx;  // into the plan's grid list, launch order (LPT)
    BatchTune tune;
    BatchTask *dev_tasks = nullptr;
    int64_t max_bytes = 0;  // size class: grids of at most this many bytes (the LDS tile of its launch)
    std::string suffix;     // timer name suffix of a size class ("" for a whole set)
};

struct PlanLarge {
    int grid = 0;
    Geom geom;
    std::vector<Step> steps;
    std::vector<Step> steps_out;  // relative plans: the out-of-place schedule
};

// Grids of a plan too large for one LDS tile but small enough that one
// workgroup transforms each of them in passes through its tile (MedTask).
struct MedGroup {
    int dtype = SGH_F64;
    std::vector<int> grid_idx;  // largest first
    MedTask *dev_tasks = nullptr;
};

int batch_lds_limit(int dtype) { return dtype == SGH_F64 ? 8192 * 8 : 16384 * 4; }

// A plan hands grids of at most g_medium_max points to the medium kernel when
// it holds at least g_medium_min of them (of one element type); fewer go out
// as per-grid launches, which then run at full-chip bandwidth each.
int64_t g_medium_max = int64_t(1) << 18;
int g_medium_min = 16;

// Size classes of the batch launch.  One launch sizes its workgroups and LDS
// tile for its largest grid, so a set of grids of very different sizes runs
// its small grids with mostly idle lanes and few workgroups per CU.  A set of
// at least g_class_min_grids grids of one dtype is split into classes by LDS
// bytes (up to 8, 16, 32, 64 KiB), one launch each; a class of fewer than
// g_class_min_per grids joins the next larger one.  Smaller sets stay one
// launch (each class launch would be too short to fill the GPU).
int g_class_min_grids = 4096;
int g_class_min_per = 1024;
int g_class_streams = 0;  // 1: class launches after the first on forked streams (measured no faster)

// Can one workgroup take grid g in passes through its tile?  Fills the task:
// after the tile pass, runs of consecutive axes share one box pass while the
// box keeps rows of at least 128 bytes (or every column of the run's stride).
bool medium_task(const Geom &g, MedTask *t) {
    if (g.N > g_medium_max) return false;
    const int64_t cap = kMedTileBytes / static_cast<int64_t>(esize_of(g.dtype));
    int m = 0;
    int64_t Sm = 1;
    while (m < g.d && Sm * g.n[m] <= cap) {
        Sm *= g.n[m];
        ++m;
    }
    if (m < 1 || m >= g.d) return false;
    for (int k = m; k < g.d; ++k)
        if (g.n[k] > cap) return false;
    if (!t) return true;
    *t = MedTask{};
    t->data = g.data;
    t->N = g.N;
    t->m = m;
    t->chunk = static_cast<int32_t>((cap / Sm) * Sm);
    t->tile = make_tile_geom(g, m);
    for (int k = 0; k < g.d; ++k) {
        t->L[k] = g.L[k];
        t->n[k] = static_cast<int32_t>(g.n[k]);
        t->st[k] = g.st[k];
    }
    // widest power-of-two column count for R rows at stride S
    auto width = [&](int64_t R, int64_t S) {
        int64_t W = 1;
        while (2 * W * R <= cap && W < S) W *= 2;
        return W;
    };
    const int64_t min_w = 128 / static_cast<int64_t>(esize_of(g.dtype));
    int k = m;
    while (k < g.d) {
        const int64_t S = g.st[k];
        int64_t R = g.n[k];
        int k1 = k + 1;
        while (k1 < g.d && R * g.n[k1] <= cap) {
            const int64_t W = width(R * g.n[k1], S);
            if (W < min_w && W < S) break;
            R *= g.n[k1];
            ++k1;
        }
        const int p = t->npass++;
        t->k0[p] = k;
        t->k1[p] = k1;
        t->W[p] = static_cast<int32_t>(width(R, S));
        k = k1;
    }
    return true;
}

void batch_default_tune(const DevInfo &di, int maxN, int ntasks, int dtype, BatchTune *t, int nt_pref = 0,
                        int persist = -1) {
    // default (what the autotuner picks on MI355X for combination sets): about
    // 16 elements per thread, 128 to 1024 threads
    int nt = nt_pref;
    if (!nt) {
        const int per = 16;
        nt = std::min(1024, std::max(128, pow2_ceil((maxN + per - 1) / per)));
        if (nt == 1024 && pow2_ceil((maxN + 1023) / 1024) > 8) nt = 512;  // 1024 threads: at most 8 each
    }
    int ept = pow2_ceil((maxN + nt - 1) / nt);
    if (ept < 4) ept = 4;
    while (ept > 32) {
        nt *= 2;
        ept = pow2_ceil((maxN + nt - 1) / nt);
        if (ept < 4) ept = 4;
    }
    t->nt = nt;
    t->ept = ept;
    t->cus = di.cus;
    t->lds_bytes = std::max<int>(static_cast<int>(maxN * esize_of(dtype)), 16);
    // resident workgroups per CU, bounded by LDS and by waves
    const int by_lds = std::max(1, di.lds_per_cu / t->lds_bytes);
    const int by_waves = std::max(1, 32 / (nt / 64));
    const int resident = std::min({by_lds, by_waves, 8}) * di.cus;
    // default: one workgroup per grid (the dispatcher balances the load) until
    // there are several grids per resident workgroup; then each resident
    // workgroup takes every nwg-th grid and prefetches the next one
    t->persist = persist >= 0 ? persist : (ntasks > 4 * resident ? 1 : 0);
    t->nwg = std::max(1, t->persist ? std::min(ntasks, resident) : ntasks);
}

}  // namespace

int report_error(int code, const char *msg) { return fail(code, "%s", msg); }

LaunchTimer::LaunchTimer(const char *name, hipStream_t s) : impl_(new TimerScope(name, s)) {}
LaunchTimer::~LaunchTimer() { delete static_cast<TimerScope *>(impl_); }
}  // namespace sgh

struct sgh_plan {
    int op = 0;
    uint32_t flags = 0;
    bool relative = false;  // grid data fields are byte offsets into the buffer given at execute
    // size classes after the first run on their own streams, forked from and
    // joined back to the caller's stream (their launches overlap)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    int64_t extent = 0;     // relative plans: bytes from offset 0 to the end of the last grid
    std::vector<sgh_grid> grids;
    std::vector<sgh::BatchGroup> groups;
    std::vector<sgh::MedGroup> medium;
    std::vector<sgh::PlanLarge> large;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
    int64_t points = 0;
};

namespace sgh {
namespace {

void fill_tasks(const sgh_plan &p, const BatchGroup &bg, std::vector<BatchTask> *tasks) {
    tasks->clear();
    for (int gi : bg.grid_idx) {
        Geom g = make_geom(p.grids[gi]);
        BatchTask t{};
        t.data = g.data;
        t.N = static_cast<int32_t>(g.N);
        t.g = make_tile_geom(g, g.d);
        tasks->push_back(t);
    }
}

void fill_med_tasks(const sgh_plan &p, const MedGroup &mg, std::vector<MedTask> *tasks) {
    tasks->clear();
    for (int gi : mg.grid_idx) {
        MedTask t{};
        (void)medium_task(make_geom(p.grids[gi]), &t);
        tasks->push_back(t);
    }
}

std::string op_prefix(int op) { return op == 0 ? "hier" : op == 1 ? "dehier" : "adjoint"; }

// The batch launches of a plan (one per size class); classes after the first
// on the plan's side streams, forked from and joined back to `st`.
hipError_t plan_launch_batches(sgh_plan *p, hipStream_t st, const void *base, const void *dbase) {
    const size_t ng = p->groups.size();
    const bool forked = ng > 1 && p->side.size() + 1 >= ng;
    if (forked) {
        hipError_t e = hipEventRecord(p->fork, st);
        if (e != hipSuccess) return e;
    }
    for (size_t i = 0; i < ng; ++i) {
        auto &bg = p->groups[i];
        hipStream_t s = (forked && i > 0) ? p->side[i - 1] : st;
        if (forked && i > 0) {
            hipError_t e = hipStreamWaitEvent(s, p->fork, 0);
            if (e != hipSuccess) return e;
        }
        {
            TimerScope ts(op_prefix(p->op) + (bg.dtype == SGH_F64 ? "_f64" : "_f32") + "_batch" + bg.suffix, s);
            hipError_t e = launch_batch(p->op, bg.dtype, bg.dev_tasks, static_cast<int32_t>(bg.grid_idx.size()),
                                        bg.tune, base, dbase, s);
            if (e != hipSuccess) return e;
        }
        if (forked && i > 0) {
            hipError_t e = hipEventRecord(p->joins[i - 1], s);
            if (e == hipSuccess) e = hipStreamWaitEvent(st, p->joins[i - 1], 0);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// A relative plan out of place: the grids at src + offset are transformed into
// dst + offset.  The batch launches read src and write dst; with medium grids
// the whole extent is copied first and those run in place on dst; large grids
// run their out-of-place schedules.
hipError_t plan_launch_out(sgh_plan *p, hipStream_t st, const void *src, void *dst) {
    if (!p->medium.empty()) {
        hipError_t e = hipMemcpyAsync(dst, src, static_cast<size_t>(p->extent), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    {
        hipError_t e = plan_launch_batches(p, st, src, dst);
        if (e != hipSuccess) return e;
    }
    for (auto &mg : p->medium) {
        TimerScope ts(op_prefix(p->op) + (mg.dtype == SGH_F64 ? "_f64" : "_f32") + "_medium", st);
        hipError_t e =
            launch_medium(p->op, mg.dtype, mg.dev_tasks, static_cast<int32_t>(mg.grid_idx.size()), dst, st);
        if (e != hipSuccess) return e;
    }
    for (auto &lg : p->large) {
        const uintptr_t off = reinterpret_cast<uintptr_t>(p->grids[lg.grid].data);
        char *d = static_cast<char *>(dst) + off;
        hipError_t e;
        if (p->medium.empty()) {
            e = run_schedule_out(p->op, lg.geom.dtype, lg.steps_out, const_cast<char *>(static_cast<const char *>(src)) + off,
                                 d, static_cast<size_t>(lg.geom.N) * esize_of(lg.geom.dtype), st);
        } else {
            std::vector<Step> steps = lg.steps;  // already copied: in place on dst
            retarget(steps, d);
            e = hipSuccess;
            for (auto &s : steps) {
                e = run_step(p->op, lg.geom.dtype, s, st);
                if (e != hipSuccess) break;
            }
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Every launch of a plan on `st`; base is null, or the buffer a relative
// plan's offsets point into.
hipError_t plan_launch_all(sgh_plan *p, hipStream_t st, const void *base = nullptr) {
    hipError_t e0 = plan_launch_batches(p, st, base, base);
    if (e0 != hipSuccess) return e0;
    for (auto &mg : p->medium) {
        TimerScope ts(op_prefix(p->op) + (mg.dtype == SGH_F64 ? "_f64" : "_f32") + "_medium", st);
        hipError_t e =
            launch_medium(p->op, mg.dtype, mg.dev_tasks, static_cast<int32_t>(mg.grid_idx.size()), base, st);
        if (e != hipSuccess) return e;
    }
    for (auto &lg : p->large) {
        if (base) {
            // one-shot launches carry their grid's address: rebased copies
            std::vector<Step> steps = lg.steps;
            retarget(steps, static_cast<char *>(const_cast<void *>(base)) +
                                reinterpret_cast<uintptr_t>(p->grids[lg.grid].data));
            for (auto &s : steps) {
                hipError_t e = run_step(p->op, lg.geom.dtype, s, st);
                if (e != hipSuccess) return e;
            }
            continue;
        }
        for (auto &s : lg.steps) {
            hipError_t e = run_step(p->op, lg.geom.dtype, s, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

int plan_capture(sgh_plan *p) {
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    if (!p->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    }
    hipError_t e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = plan_launch_all(p, p->capture_stream);
    e = hipStreamEndCapture(p->capture_stream, &p->graph);
    if (le != hipSuccess) return hip_fail(le, "launch during capture");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return SGH_OK;
}

// Time (ms) of one run of fn on a private stream: the fastest of `reps`
// samples, each the mean of a few back-to-back runs between two events (a
// launch of a few microseconds is otherwise lost in the events' own cost).
template <typename F>
float time_best(F &&fn, hipStream_t st, int reps) {
    std::vector<float> t;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return 1e30f;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return 1e30f;
    }
    // warm up, and size the samples: short launches are repeated
    int per = 1;
    {
        (void)hipEventRecord(a, st);
        hipError_t e = fn(st);
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) reps = 0, t.assign(1, 1e30f);
        else if (ms < 0.2f) per = 8;
    }
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, st);
        hipError_t e = hipSuccess;
        for (int i = 0; i < per && e == hipSuccess; ++i) e = fn(st);
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        if (e != hipSuccess) {
            t.assign(1, 1e30f);
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms / static_cast<float>(per));
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return t.empty() ? 1e30f : *std::min_element(t.begin(), t.end());
}

// Autotune a batch group: candidate workgroup sizes, timed on a scratch copy
// of the group's shapes (the caller's data is not touched).
int autotune_group(sgh_plan *p, BatchGroup &bg) {
    const DevInfo &di = dev_info();
    std::ostringstream key;
    key << di.arch << ":batch:op" << p->op << ":dt" << bg.dtype << ":n" << bg.grid_idx.size() << ":c" << bg.max_bytes
        << ":h";
    uint64_t h = 1469598103934665603ull;
    int maxN = 0;
    int64_t total = 0;
    for (int gi : bg.grid_idx) {
        const sgh_grid &g = p->grids[gi];
        for (int k = 0; k < g.dim; ++k) h = (h ^ static_cast<uint64_t>(g.level[k] + 31 * k)) * 1099511628211ull;
        h = (h ^ 0xff) * 1099511628211ull;
        Geom ge = make_geom(g);
        maxN = std::max<int>(maxN, static_cast<int>(ge.N));
        total += ge.N;
    }
    key << std::hex << h;
    std::vector<int> cached;
    if (tune_get(key.str(), &cached) && cached.size() == 2) {
        batch_default_tune(di, maxN, static_cast<int>(bg.grid_idx.size()), bg.dtype, &bg.tune, cached[0], cached[1]);
        return SGH_OK;
    }
    const size_t es = esize_of(bg.dtype);
    void *scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, static_cast<size_t>(total) * es);
    if (e != hipSuccess) return hip_fail(e, "autotune scratch");
    (void)hipMemset(scratch, 0, static_cast<size_t>(total) * es);
    std::vector<BatchTask> tasks;
    fill_tasks(*p, bg, &tasks);
    int64_t off = 0;
    for (auto &t : tasks) {
        t.data = static_cast<char *>(scratch) + off * es;
        off += t.N;
    }
    BatchTask *dtasks = nullptr;
    e = hipMalloc(&dtasks, tasks.size() * sizeof(BatchTask));
    if (e == hipSuccess) e = hipMemcpy(dtasks, tasks.data(), tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice);
    hipStream_t st = nullptr;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    int best_nt = 256, best_persist = 0;
    float best = 1e30f;
    if (e == hipSuccess) {
        for (int nt : {128, 256, 512, 1024})
            for (int persist : {0, 1}) {
                BatchTune t;
                batch_default_tune(di, maxN, static_cast<int>(tasks.size()), bg.dtype, &t, nt, persist);
                if (t.nt != nt || (nt == 1024 && t.ept > 8)) continue;
                if (persist && t.nwg == static_cast<int>(tasks.size())) continue;  // same launch as persist = 0
                const float ms = time_best(
                    [&](hipStream_t s) {
                        return launch_batch(p->op, bg.dtype, dtasks, static_cast<int32_t>(tasks.size()), t,
                                            nullptr, nullptr, s);
                    },
                    st, 7);
                if (ms < best) {
                    best = ms;
                    best_nt = nt;
                    best_persist = persist;
                }
            }
    }
    if (st) (void)hipStreamDestroy(st);
    if (dtasks) (void)hipFree(dtasks);
    (void)hipFree(scratch);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    batch_default_tune(di, maxN, static_cast<int>(bg.grid_idx.size()), bg.dtype, &bg.tune, best_nt, best_persist);
    tune_put(key.str(), {best_nt, best_persist});
    return SGH_OK;
}

// Autotune the schedule of one large grid: tile chunk multiplier and pole
// block spans, each timed alone on a scratch grid of the same shape.
bool autotune_verbose() {
    const char *v = std::getenv("SGH_AUTOTUNE_VERBOSE");
    return v && *v && *v != '0';
}

int autotune_large(sgh_plan *p, PlanLarge &lg) {
    const bool verbose = autotune_verbose();
    const std::string key = grid_key(p->op, lg.geom);
    std::vector<int> cached;
    if (tune_get(key, &cached)) {
        lg.steps = build_schedule(p->op, lg.geom);
        if (p->relative) lg.steps_out = build_schedule(p->op, lg.geom, true);
        return SGH_OK;
    }
    const size_t es = esize_of(lg.geom.dtype);
    void *scratch = nullptr;
    hipError_t e = hipMalloc(&scratch, static_cast<size_t>(lg.geom.N) * es);
    if (e != hipSuccess) return hip_fail(e, "autotune scratch");
    (void)hipMemset(scratch, 0, static_cast<size_t>(lg.geom.N) * es);
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    SchedOpts best_opts;
    float best_total = 1e30f;
    if (e == hipSuccess) {
        Geom sg = lg.geom;
        sg.data = scratch;
        std::vector<std::pair<int, bool>> walks;
        for (int w : walk_candidates(sg)) {
            walks.push_back({w, false});
            walks.push_back({w, true});  // two-level walk, where both exist
        }
        walks.push_back({-2, false});  // no fused walk
        for (auto wv : walks) {
            const int walk = wv.first;
            SchedOpts o;
            o.walk = walk;
            o.walk_two_level = wv.second;
            if (wv.second) {
                int64_t Sm = 1;
                const int m = tile_axes(sg, &Sm);
                const int L = sg.L[walk];
                const int ept = Sm <= kTWThreads ? 1 : (Sm <= 2 * kTWThreads ? 2 : 4);
                (void)m;
                // the two-level trial only differs where the three-level walk is the default
                if (!(ept == 1 && tw3_supported(L, L - 6, 3)) || !tw_supported(L, default_tw_B(L), ept)) continue;
            }
            o.pole_code.assign(static_cast<size_t>(sg.d), 0);
            auto base = build_schedule_opts(p->op, sg, o);
            for (auto &s : base) {
                if (s.kind == Step::TILE && s.tile.g.m < sg.d) {
                    int64_t Sm = 1;
                    for (int k = 0; k < s.tile.g.m; ++k) Sm *= sg.n[k];
                    float best = 1e30f;
                    for (int mult : {1, 2, 4, 8, 16}) {
                        if (Sm * mult > tile_capacity(sg.dtype)) break;
                        Step c = s;
                        c.tile.chunk = static_cast<int32_t>(Sm * mult);
                        choose_tile_tune(c.tile.chunk, &c.ttune);
                        const float ms =
                            time_best([&](hipStream_t x) { return run_step(p->op, sg.dtype, c, x); }, st, 3);
                        if (verbose)
                            std::fprintf(stderr, "[sgh autotune] %s tile m=%d chunk=%d: %.4f ms\n", key.c_str(),
                                         s.tile.g.m, c.tile.chunk, ms);
                        if (ms < best) {
                            best = ms;
                            o.tile_mult = mult;
                        }
                    }
                } else if (s.kind == Step::POLE && pole_B_override(s.pole.L) == 0 && pole3_override(s.pole.L) == 0) {
                    float best = 1e30f;
                    auto trial = [&](Step c, int code, const char *what) {
                        const float ms =
                            time_best([&](hipStream_t x) { return run_step(p->op, sg.dtype, c, x); }, st, 3);
                        if (verbose)
                            std::fprintf(stderr, "[sgh autotune] %s axis %d pole L=%d %s B=%d TB=%d pf=%d nt=%d: %.4f ms\n",
                                         key.c_str(), s.key, s.pole.L, what, c.pole.B, c.pole.TB, c.pole.pf,
                                         c.ptune.nt, ms);
                        if (ms < best) {
                            best = ms;
                            o.pole_code[static_cast<size_t>(s.key)] = code;
                        }
                    };
                    for (int B = 2; B <= s.pole.L; ++B) {
                        if (!pole_supported(s.pole.L, B)) continue;
                        for (int nt : {128, 256, 512}) {
                            Step c = s;
                            c.pole.split = 2;
                            c.pole.TB = 0;
                            c.pole.pf = 0;
                            c.pole.B = B;
                            c.ptune.nt = nt;
                            trial(c, pole_code2(B, nt), "2-level");
                        }
                    }
                    for (int TB = 0; TB <= 6; ++TB)
                        for (int B = 2; B <= 5; ++B) {
                            if (!pole3_supported(s.pole.L, TB, B)) continue;
                            for (int pf = 0; pf <= 1; ++pf) {
                                Step c = s;
                                c.pole.split = 3;
                                c.pole.TB = TB;
                                c.pole.B = B;
                                c.pole.pf = pf;
                                c.ptune.nt = 256;
                                trial(c, pole_code3(TB, B, pf, 256), "3-level");
                            }
                        }
                }
            }
            auto steps = build_schedule_opts(p->op, sg, o);
            const float total = time_best(
                [&](hipStream_t x) {
                    for (auto &s : steps) {
                        hipError_t r = run_step(p->op, sg.dtype, s, x);
                        if (r != hipSuccess) return r;
                    }
                    return hipSuccess;
                },
                st, 5);
            if (verbose)
                std::fprintf(stderr, "[sgh autotune] %s walk=%d%s schedule: %.4f ms\n", key.c_str(), walk,
                             wv.second ? " (2-level)" : "", total);
            if (total < best_total) {
                best_total = total;
                best_opts = o;
            }
        }
    }
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(scratch);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    tune_put(key, tuned_from_opts(lg.geom, best_opts));
    lg.steps = build_schedule(p->op, lg.geom);
    if (p->relative) lg.steps_out = build_schedule(p->op, lg.geom, true);
    return SGH_OK;
}

void plan_free(sgh_plan *p) {
    for (auto &bg : p->groups) {
        if (bg.dev_tasks) (void)hipFree(bg.dev_tasks);
    }
    for (auto s : p->side) (void)hipStreamDestroy(s);
    for (auto e : p->joins) (void)hipEventDestroy(e);
    if (p->fork) (void)hipEventDestroy(p->fork);
    for (auto &mg : p->medium) {
        if (mg.dev_tasks) (void)hipFree(mg.dev_tasks);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

int plan_upload(sgh_plan *p) {
    for (auto &bg : p->groups) {
        std::vector<BatchTask> tasks;
        fill_tasks(*p, bg, &tasks);
        hipError_t e = hipMemcpy(bg.dev_tasks, tasks.data(), tasks.size() * sizeof(BatchTask), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "task upload");
    }
    for (auto &mg : p->medium) {
        std::vector<MedTask> tasks;
        fill_med_tasks(*p, mg, &tasks);
        hipError_t e = hipMemcpy(mg.dev_tasks, tasks.data(), tasks.size() * sizeof(MedTask), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "task upload");
    }
    for (auto &lg : p->large) {
        lg.geom.data = p->grids[lg.grid].data;
        retarget(lg.steps, lg.geom.data);
    }
    return SGH_OK;
}

}  // namespace

int max_lds_bytes() { return dev_info().max_lds_block; }

}  // namespace sgh

// ---------------------------------------------------------------------------
// Batched transform that allocates nothing: the task list of the batch launch
// lives in a file-scope device array (each device holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel; it
// passes the device address hipGetSymbolAddress returns for the current
// device, looked up once per device.
namespace sgh {
constexpr int kStaticTasks = SGH_STATIC_TASKS;  // grids per call that the batch launch takes
constexpr int kMaxDevices = 64;
}  // namespace sgh

static __device__ __align__(256) sgh::BatchTask scratch[sgh::kStaticTasks];

namespace sgh {
namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SGH_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return SGH_OK;
}

int transform_batch_static(int op, const sgh_grid *grids, int32_t n, void *stream) {
    if (op < 0 || op > 2) return fail(SGH_ERR_ARG, "unknown op %d", op);
    int rc = validate_all(grids, n);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // grids that fit one workgroup's LDS go to the batch launch (largest
    // first, one group per dtype); the others get their own launches
    std::vector<std::pair<int64_t, int>> small[2];
    std::vector<int> large;
    for (int i = 0; i < n; ++i) {
        const Geom g = make_geom(grids[i]);
        if (g.d == 0) continue;
        if (g.N * static_cast<int64_t>(esize_of(g.dtype)) <= batch_lds_limit(g.dtype))
            small[g.dtype].push_back({g.N, i});
        else
            large.push_back(i);
    }
    const size_t ntasks = small[0].size() + small[1].size();
    if (ntasks > static_cast<size_t>(kStaticTasks))
        return fail(SGH_ERR_UNSUPPORTED, "%zu grids fit the batch tile; this entry point takes at most %d", ntasks,
                    kStaticTasks);
    std::vector<std::vector<Step>> steps(large.size());
    for (size_t j = 0; j < large.size(); ++j) {
        steps[j] = build_schedule(op, make_geom(grids[large[j]]));
        for (auto &s : steps[j])
            if (!step_launchable(s))
                return fail(SGH_ERR_UNSUPPORTED, "grid %d: no %s kernel for this shape under the current tuning knobs",
                            large[j], step_name(s));
    }
    void *dev = nullptr;
    rc = scratch_address(&dev);
    if (rc) return rc;
    if (ntasks) {
        thread_local std::vector<BatchTask> host;
        host.clear();
        for (int dt = 0; dt < 2; ++dt) {
            auto &v = small[dt];
            std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
            for (auto &x : v) {
                const Geom g = make_geom(grids[x.second]);
                BatchTask t{};
                t.data = g.data;
                t.N = static_cast<int32_t>(g.N);
                t.g = make_tile_geom(g, g.d);
                host.push_back(t);
            }
        }
        hipError_t e = hipMemcpyAsync(dev, host.data(), host.size() * sizeof(BatchTask), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "task upload");
        const DevInfo &di = dev_info();
        size_t first = 0;
        for (int dt = 0; dt < 2; ++dt) {
            if (small[dt].empty()) continue;
            BatchTune tune;
            batch_default_tune(di, static_cast<int>(small[dt].front().first), static_cast<int>(small[dt].size()), dt,
                               &tune);
            e = launch_batch(op, dt, static_cast<BatchTask *>(dev) + first, static_cast<int32_t>(small[dt].size()),
                             tune, nullptr, nullptr, st);
            if (e != hipSuccess) return hip_fail(e, "batch launch");
            first += small[dt].size();
        }
    }
    for (size_t j = 0; j < large.size(); ++j)
        for (auto &s : steps[j]) {
            hipError_t e = run_step(op, grids[large[j]].dtype, s, st);
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
        }
    return SGH_OK;
}

}  // namespace
}  // namespace sgh

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

int sgh_transform_batch_static(int32_t op, const sgh_grid *grids, int32_t n, void *stream) {
    return sgh::transform_batch_static(op, grids, n, stream);
}

int sgh_hierarchize(const sgh_grid *grids, int32_t n, void *stream) {
    return sgh::transform(SGH_OP_HIERARCHIZE, grids, n, stream);
}

int sgh_dehierarchize(const sgh_grid *grids, int32_t n, void *stream) {
    return sgh::transform(SGH_OP_DEHIERARCHIZE, grids, n, stream);
}

int sgh_hierarchize_adjoint(const sgh_grid *grids, int32_t n, void *stream) {
    return sgh::transform(SGH_OP_ADJOINT, grids, n, stream);
}

int sgh_transform(int32_t op, const sgh_grid *grids, int32_t n, void *stream) {
    return sgh::transform(op, grids, n, stream);
}

int sgh_transform_out(int32_t op, const sgh_grid *src, const sgh_grid *dst, int32_t n, void *stream) {
    return sgh::transform_out(op, src, dst, n, stream);
}

int sgh_validate(const sgh_grid *grids, int32_t n) { return sgh::validate_all(grids, n); }

int64_t sgh_num_points(const sgh_grid *grid) {
    if (!grid) return -1;
    sgh_grid g = *grid;
    if (g.data == nullptr) g.data = reinterpret_cast<void *>(uintptr_t(256));  // size query only
    int64_t n = 0;
    if (sgh::validate_one(g, 0, &n) != SGH_OK) return -1;
    return n;
}

int sgh_schedule_describe(int32_t op, const sgh_grid *grid, char *buf, int32_t len) {
    if (!grid || op < 0 || op > 2) return sgh::fail(SGH_ERR_ARG, "bad arguments");
    sgh_grid g = *grid;
    if (g.data == nullptr) g.data = reinterpret_cast<void *>(uintptr_t(256));
    int64_t np = 0;
    int rc = sgh::validate_one(g, 0, &np);
    if (rc) return rc;
    sgh::Geom ge = sgh::make_geom(g);
    return sgh::copy_out(sgh::describe_steps(op, ge, sgh::build_schedule(op, ge)), buf, len);
}

int sgh_schedule_describe_out(int32_t op, const sgh_grid *grid, char *buf, int32_t len) {
    if (!grid || op < 0 || op > 2) return sgh::fail(SGH_ERR_ARG, "bad arguments");
    sgh_grid g = *grid;
    if (g.data == nullptr) g.data = reinterpret_cast<void *>(uintptr_t(256));
    int64_t np = 0;
    int rc = sgh::validate_one(g, 0, &np);
    if (rc) return rc;
    sgh::Geom ge = sgh::make_geom(g);
    return sgh::copy_out(sgh::describe_steps(op, ge, sgh::build_schedule(op, ge, true)), buf, len);
}

const char *sgh_error_string(int code) {
    switch (code) {
        case SGH_OK: return "success";
        case SGH_ERR_ARG: return "invalid argument";
        case SGH_ERR_DTYPE: return "invalid dtype";
        case SGH_ERR_ALIGN: return "misaligned data pointer";
        case SGH_ERR_OVERLAP: return "grids overlap";
        case SGH_ERR_HIP: return "HIP runtime error";
        case SGH_ERR_NOMEM: return "out of memory";
        case SGH_ERR_UNSUPPORTED: return "unsupported request";
        default: return "unknown error";
    }
}

const char *sgh_last_error_message(void) { return sgh::g_last_error.c_str(); }

const char *sgh_version(void) { return "0.1.0"; }

int sgh_plan_create(sgh_plan **plan, int32_t op, const sgh_grid *grids, int32_t n, uint32_t flags) {
    using namespace sgh;
    if (!plan) return fail(SGH_ERR_ARG, "null plan pointer");
    *plan = nullptr;
    if (op < 0 || op > 2) return fail(SGH_ERR_ARG, "unknown op %d", op);
    if (flags & ~(SGH_PLAN_GRAPH | SGH_PLAN_AUTOTUNE | SGH_PLAN_RELATIVE))
        return fail(SGH_ERR_ARG, "unknown plan flags 0x%x", flags);
    const bool relative = (flags & SGH_PLAN_RELATIVE) != 0;
    int rc = validate_all(grids, n, relative);
    if (rc) return rc;
    std::unique_ptr<sgh_plan, void (*)(sgh_plan *)> p(new (std::nothrow) sgh_plan, plan_free);
    if (!p) return fail(SGH_ERR_NOMEM, "plan allocation");
    p->op = op;
    p->flags = flags;
    p->relative = relative;
    p->grids.assign(grids, grids + n);
    const DevInfo &di = dev_info();
    // split: grids that fit one workgroup's LDS go to the batch kernel
    std::map<int, std::vector<std::pair<int64_t, int>>> small, medium;
    std::vector<int> large;
    for (int i = 0; i < n; ++i) {
        Geom g = make_geom(grids[i]);
        p->points += g.N;
        if (relative)
            p->extent = std::max<int64_t>(p->extent, static_cast<int64_t>(reinterpret_cast<uintptr_t>(grids[i].data)) +
                                                         g.N * static_cast<int64_t>(esize_of(g.dtype)));
        if (g.d == 0) continue;  // all axes of level 1: identity
        if (g.N * static_cast<int64_t>(esize_of(g.dtype)) <= batch_lds_limit(g.dtype))
            small[g.dtype].push_back({g.N, i});
        else if (medium_task(g, nullptr))
            medium[g.dtype].push_back({g.N, i});
        else
            large.push_back(i);
    }
    for (auto &kv : medium) {
        auto v = kv.second;
        if (static_cast<int>(v.size()) < g_medium_min) {
            for (auto &x : v) large.push_back(x.second);
            continue;
        }
        std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        MedGroup mg;
        mg.dtype = kv.first;
        for (auto &x : v) mg.grid_idx.push_back(x.second);
        hipError_t e = hipMalloc(&mg.dev_tasks, v.size() * sizeof(MedTask));
        if (e != hipSuccess) return hip_fail(e, "task list");
        p->medium.push_back(mg);
    }
    std::sort(large.begin(), large.end());
    for (int i : large) {
        PlanLarge lg;
        lg.grid = i;
        lg.geom = make_geom(grids[i]);
        lg.steps = build_schedule(op, lg.geom);
        if (relative) lg.steps_out = build_schedule(op, lg.geom, true);
        p->large.push_back(lg);
    }
    int class_min_grids, class_min_per;
    {
        std::lock_guard<std::mutex> lk(g_override_mu);
        class_min_grids = g_class_min_grids;
        class_min_per = g_class_min_per;
    }
    for (auto &kv : small) {
        auto v = kv.second;
        const int dtype = kv.first;
        const int64_t es = static_cast<int64_t>(esize_of(dtype));
        // longest processing time first; ties keep list order
        std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        std::vector<std::pair<int64_t, std::vector<std::pair<int64_t, int>>>> classes;
        if (class_min_grids > 0 && static_cast<int>(v.size()) >= class_min_grids) {
            const int64_t bounds[] = {8192, 16384, 32768, 65536};
            for (int64_t b : bounds) classes.push_back({b, {}});
            for (auto &x : v) {
                size_t c = 0;
                while (x.first * es > classes[c].first) ++c;
                classes[c].second.push_back(x);
            }
            // small classes join the next larger one (largest grids stay first)
            for (size_t c = 0; c + 1 < classes.size(); ++c)
                if (!classes[c].second.empty() && static_cast<int>(classes[c].second.size()) < class_min_per) {
                    auto &nx = classes[c + 1].second;
                    nx.insert(nx.end(), classes[c].second.begin(), classes[c].second.end());
                    classes[c].second.clear();
                }
            // largest class first, so that its long grids start early
            std::reverse(classes.begin(), classes.end());
        } else {
            classes.push_back({0, v});
        }
        for (auto &cl : classes) {
            if (cl.second.empty()) continue;
            BatchGroup bg;
            bg.dtype = dtype;
            bg.max_bytes = cl.first;
            if (cl.first) bg.suffix = "_c" + std::to_string(cl.first / 1024) + "k";
            for (auto &x : cl.second) bg.grid_idx.push_back(x.second);
            const int maxN = static_cast<int>(cl.second.front().first);
            batch_default_tune(di, maxN, static_cast<int>(cl.second.size()), bg.dtype, &bg.tune);
            hipError_t e = hipMalloc(&bg.dev_tasks, cl.second.size() * sizeof(BatchTask));
            if (e != hipSuccess) return hip_fail(e, "task list");
            p->groups.push_back(bg);
        }
    }
    if (p->groups.size() > 1 && g_class_streams) {
        hipError_t e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        for (size_t i = 1; e == hipSuccess && i < p->groups.size(); ++i) {
            hipStream_t s = nullptr;
            hipEvent_t j = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
            if (e == hipSuccess) p->side.push_back(s);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
            if (e == hipSuccess) p->joins.push_back(j);
        }
        if (e != hipSuccess) return hip_fail(e, "class streams");
    }
    if (flags & SGH_PLAN_AUTOTUNE) {
        for (auto &bg : p->groups) {
            rc = autotune_group(p.get(), bg);
            if (rc) return rc;
        }
        for (auto &lg : p->large) {
            rc = autotune_large(p.get(), lg);
            if (rc) return rc;
        }
    }
    for (const auto &lg : p->large)
        for (const auto *v : {&lg.steps, &lg.steps_out})
            for (const auto &s : *v)
                if (!step_launchable(s))
                return fail(SGH_ERR_UNSUPPORTED, "grid %d: no %s kernel for this shape under the current tuning knobs",
                            lg.grid, step_name(s));
    rc = plan_upload(p.get());
    if (rc) return rc;
    // a single launch goes out directly: replaying a one-node graph measured
    // slower than the launch it holds
    size_t launches = p->groups.size() + p->medium.size();
    for (const auto &lg : p->large) launches += lg.steps.size();
    if ((flags & SGH_PLAN_GRAPH) && launches > 1 && !relative) {
        rc = plan_capture(p.get());
        if (rc) return rc;
    }
    *plan = p.release();
    return SGH_OK;
}

int sgh_plan_execute(sgh_plan *p, void *stream) {
    using namespace sgh;
    if (!p) return fail(SGH_ERR_ARG, "null plan");
    if (p->relative) return fail(SGH_ERR_ARG, "a relative plan needs its buffer: sgh_plan_execute_at");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->exec) {
        TimerScope ts("graph", st);
        hipError_t e = hipGraphLaunch(p->exec, st);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return SGH_OK;
    }
    hipError_t e = plan_launch_all(p, st);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return SGH_OK;
}

int sgh_plan_execute_at(sgh_plan *p, void *base, void *stream) {
    using namespace sgh;
    if (!p) return fail(SGH_ERR_ARG, "null plan");
    if (!p->relative) return fail(SGH_ERR_ARG, "sgh_plan_execute_at needs a plan created with SGH_PLAN_RELATIVE");
    if (!base) return fail(SGH_ERR_ARG, "null base");
    for (const auto &g : p->grids)
        if (reinterpret_cast<uintptr_t>(base) % esize_of(g.dtype) != 0)
            return fail(SGH_ERR_ALIGN, "base %p not aligned to %zu bytes", base, esize_of(g.dtype));
    hipError_t e = plan_launch_all(p, static_cast<hipStream_t>(stream), base);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return SGH_OK;
}

int sgh_plan_execute_out(sgh_plan *p, const void *src_base, void *dst_base, void *stream) {
    using namespace sgh;
    if (!p) return fail(SGH_ERR_ARG, "null plan");
    if (!p->relative) return fail(SGH_ERR_ARG, "sgh_plan_execute_out needs a plan created with SGH_PLAN_RELATIVE");
    if (!src_base || !dst_base) return fail(SGH_ERR_ARG, "null base");
    for (const auto &g : p->grids)
        if (reinterpret_cast<uintptr_t>(src_base) % esize_of(g.dtype) != 0 ||
            reinterpret_cast<uintptr_t>(dst_base) % esize_of(g.dtype) != 0)
            return fail(SGH_ERR_ALIGN, "base not aligned to %zu bytes", esize_of(g.dtype));
    hipError_t e;
    if (src_base == dst_base) {
        e = plan_launch_all(p, static_cast<hipStream_t>(stream), dst_base);
    } else {
        const uintptr_t a = reinterpret_cast<uintptr_t>(src_base), b = reinterpret_cast<uintptr_t>(dst_base);
        const uintptr_t x = static_cast<uintptr_t>(p->extent);
        if (a < b + x && b < a + x) return fail(SGH_ERR_OVERLAP, "source and destination buffers overlap");
        e = plan_launch_out(p, static_cast<hipStream_t>(stream), src_base, dst_base);
    }
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return SGH_OK;
}

int sgh_plan_set_data(sgh_plan *p, const sgh_grid *grids, int32_t n) {
    using namespace sgh;
    if (!p) return fail(SGH_ERR_ARG, "null plan");
    if (n != static_cast<int32_t>(p->grids.size())) return fail(SGH_ERR_ARG, "grid count %d != plan's %zu", n, p->grids.size());
    int rc = validate_all(grids, n, p->relative);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        const sgh_grid &a = p->grids[i], &b = grids[i];
        bool same = a.dim == b.dim && a.dtype == b.dtype;
        for (int k = 0; same && k < a.dim; ++k) same = a.level[k] == b.level[k];
        if (!same) return fail(SGH_ERR_ARG, "grid %d: shape or dtype differs from the plan", i);
    }
    // the task list may still be read by an execute in flight on any stream
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    for (int i = 0; i < n; ++i) p->grids[i].data = grids[i].data;
    rc = plan_upload(p);
    if (rc) return rc;
    if (p->exec && !p->large.empty()) return plan_capture(p);  // large-grid launches carry pointers
    return SGH_OK;
}

int sgh_plan_describe(const sgh_plan *p, char *buf, int32_t len) {
    using namespace sgh;
    if (!p) return fail(SGH_ERR_ARG, "null plan");
    std::ostringstream ss;
    ss << "{\"op\":" << p->op << ",\"grids\":" << p->grids.size() << ",\"points\":" << p->points
       << ",\"graph\":" << (p->exec ? "true" : "false") << ",\"relative\":" << (p->relative ? "true" : "false")
       << ",\"batches\":[";
    for (size_t i = 0; i < p->groups.size(); ++i) {
        const auto &bg = p->groups[i];
        if (i) ss << ",";
        int64_t pts = 0;
        for (int gi : bg.grid_idx) pts += make_geom(p->grids[gi]).N;
        ss << "{\"dtype\":" << bg.dtype << ",\"tasks\":" << bg.grid_idx.size() << ",\"points\":" << pts
           << ",\"nt\":" << bg.tune.nt
           << ",\"ept\":" << bg.tune.ept << ",\"workgroups\":" << bg.tune.nwg << ",\"lds_bytes\":" << bg.tune.lds_bytes
           << ",\"persistent\":" << bg.tune.persist << ",\"class_bytes\":" << bg.max_bytes
           << "}";
    }
    ss << "],\"medium\":[";
    for (size_t i = 0; i < p->medium.size(); ++i) {
        const auto &mg = p->medium[i];
        if (i) ss << ",";
        int64_t pts = 0;
        for (int gi : mg.grid_idx) pts += make_geom(p->grids[gi]).N;
        ss << "{\"dtype\":" << mg.dtype << ",\"tasks\":" << mg.grid_idx.size() << ",\"points\":" << pts
           << ",\"tile_bytes\":" << kMedTileBytes << "}";
    }
    ss << "],\"large\":[";
    for (size_t i = 0; i < p->large.size(); ++i) {
        if (i) ss << ",";
        ss << describe_steps(p->op, p->large[i].geom, p->large[i].steps);
    }
    ss << "]}";
    return copy_out(ss.str(), buf, len);
}

void sgh_plan_destroy(sgh_plan *p) {
    if (p) sgh::plan_free(p);
}

int sgh_set_pole_block(int32_t level, int32_t block_exponent) {
    using namespace sgh;
    if (level < 2 || level > SGH_MAX_LEVEL) return fail(SGH_ERR_ARG, "level %d outside 2..%d", level, SGH_MAX_LEVEL);
    if (block_exponent != 0 && !pole_supported(level, block_exponent))
        return fail(SGH_ERR_UNSUPPORTED, "no pole kernel for level %d with block exponent %d", level, block_exponent);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_pole_B_override[level] = block_exponent;
    return SGH_OK;
}

int sgh_set_pole_split(int32_t level, int32_t top_exponent, int32_t block_exponent, int32_t prefetch) {
    using namespace sgh;
    if (level < 2 || level > SGH_MAX_LEVEL) return fail(SGH_ERR_ARG, "level %d outside 2..%d", level, SGH_MAX_LEVEL);
    if (block_exponent == 0) {
        std::lock_guard<std::mutex> lk(g_override_mu);
        g_pole3_override[level] = 0;
        return SGH_OK;
    }
    if (!pole3_supported(level, top_exponent, block_exponent) || prefetch < 0 || prefetch > 1)
        return fail(SGH_ERR_UNSUPPORTED, "no three-level pole kernel for level %d = %d + 2*%d", level, top_exponent,
                    block_exponent);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_pole3_override[level] = 1 + top_exponent * 100 + block_exponent * 10 + prefetch;
    return SGH_OK;
}

int sgh_set_walk_preference(int32_t pref) {
    using namespace sgh;
    if (pref < 0 || pref > 1) return fail(SGH_ERR_ARG, "walk preference %d outside 0..1", pref);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_walk_pref = pref;
    return SGH_OK;
}

int sgh_set_split_spans(int32_t fine, int32_t coarse) {
    using namespace sgh;
    if (fine < 0 || fine > 16 || coarse < 0 || coarse > 16)
        return fail(SGH_ERR_ARG, "split span exponents %d, %d outside 0..16", fine, coarse);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_split_fine = fine;
    g_split_coarse = coarse;
    return SGH_OK;
}

int sgh_set_box_limits(int32_t max_bytes, int32_t min_row_bytes) {
    using namespace sgh;
    if (max_bytes < 0 || max_bytes > 160 * 1024 || min_row_bytes < 0 || min_row_bytes > 512)
        return fail(SGH_ERR_ARG, "box limits %d, %d outside 0..%d, 0..512", max_bytes, min_row_bytes, 160 * 1024);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_box_bytes = max_bytes;
    g_box_row = min_row_bytes;
    return SGH_OK;
}

int sgh_set_medium_limits(int64_t max_points, int32_t min_grids) {
    using namespace sgh;
    if (max_points < 0 || max_points > (int64_t(1) << 24) || min_grids < 1)
        return fail(SGH_ERR_ARG, "medium limits %lld, %d outside 0..2^24, >= 1", static_cast<long long>(max_points),
                    min_grids);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_medium_max = max_points;
    g_medium_min = min_grids;
    return SGH_OK;
}

int sgh_set_batch_classes(int32_t min_grids, int32_t min_per_class, int32_t concurrent) {
    using namespace sgh;
    if (min_grids < 0 || min_per_class < 1 || concurrent < 0 || concurrent > 1)
        return fail(SGH_ERR_ARG, "batch class limits %d, %d, %d outside >= 0, >= 1, 0..1", min_grids, min_per_class,
                    concurrent);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_class_min_grids = min_grids;
    g_class_min_per = min_per_class;
    g_class_streams = concurrent;
    return SGH_OK;
}

int sgh_set_outer_stencil(int32_t on) {
    using namespace sgh;
    if (on < 0 || on > 1) return fail(SGH_ERR_ARG, "outer stencil switch %d outside 0..1", on);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_outer_stencil = on;
    return SGH_OK;
}

int sgh_set_xcd_order(int32_t on) {
    using namespace sgh;
    if (on < 0 || on > 1) return fail(SGH_ERR_ARG, "XCD order switch %d outside 0..1", on);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_tw_xcd = on;
    return SGH_OK;
}

int sgh_set_fusion(int32_t level) {
    using namespace sgh;
    if (level < 0 || level > 2) return fail(SGH_ERR_ARG, "fusion level %d outside 0..2", level);
    std::lock_guard<std::mutex> lk(g_override_mu);
    g_fusion = level;
    return SGH_OK;
}

int sgh_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(sgh::g_time_mu);
    sgh::g_timing = on != 0;
    return SGH_OK;
}

int sgh_timing_reset(void) {
    std::lock_guard<std::mutex> lk(sgh::g_time_mu);
    for (auto &t : sgh::g_timed) {
        (void)hipEventSynchronize(t.b);
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    sgh::g_timed.clear();
    sgh::g_time_acc.clear();
    return SGH_OK;
}

int sgh_timing_report(char *buf, int32_t len) {
    std::lock_guard<std::mutex> lk(sgh::g_time_mu);
    sgh::timing_drain_locked();
    std::ostringstream ss;
    ss << "{";
    bool first = true;
    for (auto &kv : sgh::g_time_acc) {
        if (!first) ss << ",";
        first = false;
        char num[64];
        std::snprintf(num, sizeof(num), "%.6f", kv.second.second);
        ss << "\"" << kv.first << "\":{\"count\":" << kv.second.first << ",\"ms\":" << num << "}";
    }
    ss << "}";
    return sgh::copy_out(ss.str(), buf, len);
}

}  // extern "C"
