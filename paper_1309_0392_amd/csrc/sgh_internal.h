// Internal declarations shared by the host side (sgh_api.cpp) and the
// kernels (sgh_kernels.hip) of the hierarchization library.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sgh.h"

namespace sgh {

constexpr int kMaxDim = SGH_MAX_DIM;

// Longest pole kept entirely in registers by the strided-axis kernel.  A pole
// of level L is split into 2^(L-B) dyadic blocks of span 2^B.
constexpr int kPoleMaxLevel = 10;

// Geometry of a tile transformed in LDS: the leading `m` axes (all of level
// >= 2) of a grid, viewed inside a contiguous run of elements.  Element e of
// the run has 1-based position  ((e / st[k]) % n[k]) + 1  along slab axis k.
struct TileGeom {
    int32_t m;
    int32_t L[kMaxDim];
    int32_t n[kMaxDim];
    int32_t st[kMaxDim];
    float rst[kMaxDim];  // 1 / st, for exact quotient estimates below 2^15
    float rn[kMaxDim];   // 1 / n
};

// One launch over contiguous runs ("chunks") of `chunk` elements each; every
// chunk holds whole tiles, so it is transformed independently in LDS.
struct TileLaunch {
    void *data;
    int64_t total;  // elements in the grid
    int32_t chunk;  // elements per chunk (a multiple of the tile size)
    TileGeom g;
};

// One grid of a batch, transformed whole in LDS.
struct BatchTask {
    void *data;
    int32_t N;
    int32_t pad;
    TileGeom g;
};

// The medium launch's tile (bytes of LDS per workgroup), elements per thread
// (FP64, FP32; the workgroup size follows), and whether the next step's
// values are loaded while the current step is transformed.
#ifndef SGH_MEDIUM_TILE_BYTES
#define SGH_MEDIUM_TILE_BYTES 65536
#endif
#ifndef SGH_MEDIUM_EPT64
#define SGH_MEDIUM_EPT64 16
#endif
#ifndef SGH_MEDIUM_EPT32
#define SGH_MEDIUM_EPT32 16
#endif
#ifndef SGH_MEDIUM_PREFETCH
#define SGH_MEDIUM_PREFETCH 1
#endif
// Minimum waves per SIMD the medium kernel is compiled for (0: the compiler's choice).
#ifndef SGH_MEDIUM_WAVES
#define SGH_MEDIUM_WAVES 0
#endif
constexpr int kMedTileBytes = SGH_MEDIUM_TILE_BYTES;
constexpr int kMedEpt64 = SGH_MEDIUM_EPT64;
constexpr int kMedEpt32 = SGH_MEDIUM_EPT32;
constexpr bool kMedPrefetch = SGH_MEDIUM_PREFETCH != 0;

// A grid of a batched plan too large for one LDS tile, transformed by one
// workgroup in passes through its tile: the leading tile axes in chunks of
// whole tiles, then runs of consecutive further axes k0..k1-1, each run in
// boxes of W adjacent columns times the run's whole extent (consecutive axes
// have strides S, S*n_k0, ..., so the box is W columns by n_k0*...*n_(k1-1)
// rows at stride S).  Inverse and transpose take the passes in reverse.
struct MedTask {
    void *data;
    int64_t N;
    int32_t m;      // leading axes of the tile pass
    int32_t chunk;  // elements per tile chunk (whole tiles)
    int32_t npass;  // box passes after the tile pass
    int32_t pad;
    TileGeom tile;  // the tile pass's axes
    int32_t L[kMaxDim];
    int32_t n[kMaxDim];
    int64_t st[kMaxDim];
    int32_t k0[kMaxDim];  // box pass p takes axes k0[p] .. k1[p]-1
    int32_t k1[kMaxDim];
    int32_t W[kMaxDim];   // columns per box of pass p, a power of two
};

// Strided axis: npoles = outer * S poles of n = 2^L - 1 points at stride S.
// split 2: blocks of span 2^B between coarse points (2^(L-B) blocks);
// split 3: 2^TB super-blocks of 2^B blocks of span 2^B (L = TB + 2B), with the
// next group of rows prefetched when pf is set.
struct PoleLaunch {
    void *data;
    void *dst = nullptr;  // destination grid (null: in place)
    int64_t npoles;
    int64_t S;
    int32_t L;
    int32_t B;
    int32_t split = 2;
    int32_t TB = 0;
    int32_t pf = 0;
};

// Leading tile axes fused with one walked strided axis: workgroup w owns the
// pencil of all tile elements over the whole walked pole, at element offset
// (w / mid) * n * Sw + (w % mid) * Sm; row p (1-based position on the walked
// axis) starts (p - 1) * Sw elements further.
struct TWLaunch {
    void *data;
    void *dst = nullptr;  // destination grid (null: in place)
    int64_t nwg;  // pencils: (N / (n * Sw)) * mid
    int64_t mid;  // Sw / Sm
    int64_t Sw;   // stride of the walked axis (elements)
    int32_t Sm;   // tile size (elements of one row)
    int32_t L;    // level of the walked axis
    int32_t B;    // block exponent along the walked axis
    int32_t ept;  // tile elements per thread (threads = 1024)
    int32_t split = 2;  // 2: two-level walk; 3: three-level walk (L = TB + 2B, ept 1)
    int32_t TB = 0;
    // Hierarchization out of place with the three-level walk only: the axis
    // right after the walked one (stride n * Sw, level oL, on = 2^oL - 1
    // points) is transformed in the same pass by its one-shot stencil, applied
    // as the rows are read (oL = 0: off).
    int32_t oL = 0;
    int32_t on = 0;
    int32_t xcd = 0;  // 1: consecutive pencils on one XCD (workgroup order)
    TileGeom g;   // tile axes
};

// Several consecutive small strided axes in one pass.  A workgroup loads a
// box of W adjacent columns (consecutive elements below the stride S of the
// group's first axis) times the full extent of the group's axes (P points)
// into LDS, transforms the group's axes there with the tile code (the W
// columns are a batch dimension) and writes the box back.
struct BoxLaunch {
    void *data;
    int64_t S;      // stride of the group's first axis
    int64_t outer;  // total / (S * P)
    int32_t P;      // product of the group's n_k
    int32_t W;      // columns per workgroup, a power of two
    TileGeom g;     // the group's axes inside the box (strides W * prod of earlier n)
};

// One phase of the dyadic split of poles too long for one pass.  The pole
// positions p = t * 2^E (t = 1 .. 2^(L-E) - 1, the "lattice" of this phase)
// are cut into blocks of 2^Bs lattice steps; a workgroup loads one block of
// W adjacent poles together with the two block-boundary positions (zero at
// t = 0 and t = 2^(L-E)) and applies the 1-D rule for the levels inside the
// block, which only involve the block and its boundaries.  The boundaries
// are the next phase's lattice (E + Bs).  Hierarchization runs the phases
// fine to coarse, the inverse and the transpose coarse to fine; the transpose
// also takes, for each interior point of a phase with E > 0, its children
// finer than the lattice (distances 2^(E-1) .. 1).
struct SplitLaunch {
    void *data;
    int64_t S;      // elements between consecutive positions of a pole
    int64_t outer;  // pole groups of S adjacent poles; group o starts at o * (2^L - 1) * S
    int32_t L;      // pole level
    int32_t E;      // lattice exponent
    int32_t Bs;     // block span exponent along the lattice
    int32_t W;      // adjacent poles per workgroup, a power of two <= 64
};

// Largest block span exponent of a split phase with W poles per workgroup
// (the tile of W * (2^Bs + 1) elements stays within 64 KiB plus one row).
inline int split_max_span(int W, int esize) {
    int b = 1;
    while (static_cast<int64_t>(W) * esize << (b + 1) <= 65536) ++b;
    return b;
}

struct TileTune {
    int nt = 256;   // threads per workgroup
    int ept = 4;    // elements per thread (chunk <= nt * ept)
    int grid = 0;   // workgroups (0 = one per chunk)
};

struct PoleTune {
    int nt = 256;
};

struct BatchTune {
    int nt = 256;
    int ept = 8;
    int nwg = 0;        // one workgroup per grid, or the resident count (each then owns several grids)
    int lds_bytes = 0;
    int persist = 0;    // 1: nwg = resident workgroups (capped at launch by the kernel's occupancy)
    int cus = 256;      // compute units of the device
};

// Launchers per element type and operation (return the first HIP error,
// hipSuccess otherwise).
#define SGH_DECLARE_LAUNCHERS(SUF)                                                                    \
    hipError_t launch_tile_##SUF(const TileLaunch &p, const TileTune &t, hipStream_t s);              \
    hipError_t launch_pole_##SUF(const PoleLaunch &p, const PoleTune &t, hipStream_t s);              \
    hipError_t launch_tw_##SUF(const TWLaunch &p, hipStream_t s);                                     \
    hipError_t launch_split_##SUF(const SplitLaunch &p, hipStream_t s);                               \
    hipError_t launch_box_##SUF(const BoxLaunch &p, const TileTune &t, hipStream_t s);                \
    hipError_t launch_medium_##SUF(const MedTask *dev_tasks, int32_t ntasks, const void *base,        \
                                   hipStream_t s);                                                    \
    hipError_t launch_batch_##SUF(const BatchTask *dev_tasks, int32_t ntasks, const BatchTune &t,    \
                                  const void *base, const void *dbase, hipStream_t s);
SGH_DECLARE_LAUNCHERS(f64_h)
SGH_DECLARE_LAUNCHERS(f64_d)
SGH_DECLARE_LAUNCHERS(f64_a)
SGH_DECLARE_LAUNCHERS(f32_h)
SGH_DECLARE_LAUNCHERS(f32_d)
SGH_DECLARE_LAUNCHERS(f32_a)
#undef SGH_DECLARE_LAUNCHERS

#define SGH_ROUTE(NAME, ...)                                              \
    do {                                                                  \
        if (dtype == SGH_F64) {                                           \
            if (op == SGH_OP_HIERARCHIZE) return NAME##_f64_h(__VA_ARGS__);   \
            if (op == SGH_OP_DEHIERARCHIZE) return NAME##_f64_d(__VA_ARGS__); \
            if (op == SGH_OP_ADJOINT) return NAME##_f64_a(__VA_ARGS__);       \
        } else if (dtype == SGH_F32) {                                    \
            if (op == SGH_OP_HIERARCHIZE) return NAME##_f32_h(__VA_ARGS__);   \
            if (op == SGH_OP_DEHIERARCHIZE) return NAME##_f32_d(__VA_ARGS__); \
            if (op == SGH_OP_ADJOINT) return NAME##_f32_a(__VA_ARGS__);       \
        }                                                                 \
        return hipErrorInvalidValue;                                      \
    } while (0)

inline hipError_t launch_tile(int op, int dtype, const TileLaunch &p, const TileTune &t, hipStream_t s) {
    SGH_ROUTE(launch_tile, p, t, s);
}
inline hipError_t launch_pole(int op, int dtype, const PoleLaunch &p, const PoleTune &t, hipStream_t s) {
    SGH_ROUTE(launch_pole, p, t, s);
}
inline hipError_t launch_tw(int op, int dtype, const TWLaunch &p, hipStream_t s) { SGH_ROUTE(launch_tw, p, s); }
inline hipError_t launch_split(int op, int dtype, const SplitLaunch &p, hipStream_t s) {
    SGH_ROUTE(launch_split, p, s);
}
inline hipError_t launch_box(int op, int dtype, const BoxLaunch &p, const TileTune &t, hipStream_t s) {
    SGH_ROUTE(launch_box, p, t, s);
}
// Batch and medium task lists hold grid addresses relative to `base` (null:
// absolute device addresses); the batch launch stores relative to `dbase`
// (equal to base: in place).
inline hipError_t launch_medium(int op, int dtype, const MedTask *dev_tasks, int32_t ntasks, const void *base,
                                hipStream_t s) {
    SGH_ROUTE(launch_medium, dev_tasks, ntasks, base, s);
}
inline hipError_t launch_batch(int op, int dtype, const BatchTask *dev_tasks, int32_t ntasks, const BatchTune &t,
                               const void *base, const void *dbase, hipStream_t s) {
    SGH_ROUTE(launch_batch, dev_tasks, ntasks, t, base, dbase, s);
}
#undef SGH_ROUTE

bool pole_supported(int L, int B);
bool pole3_supported(int L, int TB, int B);
bool tw3_supported(int L, int TB, int B);
// Threads per workgroup of the fused tile + walked-axis kernel, and the
// (L, B, ept) combinations it is built for.
constexpr int kTWThreads = 1024;
bool tw_supported(int L, int B, int ept);
// LDS rows staged at once by the fused kernel: 16 / ept rows of the tile for
// the two-level walk, 8 rows for the three-level walk (groups of 7 rows, so
// two workgroups fit one CU's LDS).
constexpr int tw_rows_per_batch(int ept) { return 16 / ept; }
constexpr int kTW3Rows = 8;
bool tile_ept_supported(int ept);
bool batch_ept_supported(int ept);
int max_lds_bytes();

}  // namespace sgh

namespace sgh {

// ---------------------------------------------------------------------------
// Combination technique: gather / scatter of surpluses between the grids of a
// combination set and the sparse grid (one dtype per set).
struct CombiGrid {
    void *data;
    int32_t L[kMaxDim];
    int64_t st[kMaxDim];  // element stride per axis
    int64_t n[kMaxDim];   // points per axis
    // x / n[k] == (x * magic[k]) >> mshift[k] for 0 <= x < 2^31 (magic < 2^33)
    uint64_t magic[kMaxDim];
    int32_t mshift[kMaxDim];
};

// A work unit: 2^e consecutive points of one subspace (gather; at most
// 256), or up to 256 consecutive points of one grid (scatter).
struct CombiUnit {
    int32_t owner;  // subspace (gather) or grid (scatter)
    int32_t count;
    int64_t start;
};

// Products staged in LDS per gather chunk (pairs of point and contributor).
constexpr int kCombiPairs = 2048;

struct CombiLaunch {
    int32_t d;
    int32_t nunits;
    const CombiGrid *grids;        // [ngrids]
    const int32_t *sub_levels;     // [nsub * d]
    const int64_t *sub_offsets;    // [nsub]
    const int32_t *contrib_begin;  // [nsub + 1], gather: contributors of subspace s, grid-list order
    const int64_t *contrib_addr;   // byte address of the contributor's data minus sum_k st_k elements
    const int64_t *contrib_mul;    // [ncontrib * d]: elements per odd-index step, 2^(L_k - m_k) * st_k
    const double *contrib_coef;    // coefficient per contributor
    const int64_t *table;          // scatter: subspace offset by level vector, dense
    int64_t tstride[kMaxDim];      // scatter: table stride per axis (levels 1..maxL)
    int32_t fast32;                // scatter: every grid has fewer than 2^31 points
    const CombiUnit *units;
    void *sparse;
};

// Records `msg` as the library's last error message; returns `code`.
int report_error(int code, const char *msg);

// Brackets the launches made on `s` during its lifetime with timing events
// while sgh_timing_enable is on (reported under `name`).
class LaunchTimer {
public:
    LaunchTimer(const char *name, hipStream_t s);
    ~LaunchTimer();
    LaunchTimer(const LaunchTimer &) = delete;
    LaunchTimer &operator=(const LaunchTimer &) = delete;

private:
    void *impl_;
};

hipError_t launch_combi_gather_f64(const CombiLaunch &p, hipStream_t s);
hipError_t launch_combi_gather_f32(const CombiLaunch &p, hipStream_t s);
hipError_t launch_combi_scatter_f64(const CombiLaunch &p, hipStream_t s);
hipError_t launch_combi_scatter_f32(const CombiLaunch &p, hipStream_t s);

}  // namespace sgh
