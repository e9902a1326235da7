// htree_dev.h -- device data structures and launch wrappers shared by the
// HIP translation units of libhtree (gfx950, wave64).
//
// A context holds S >= 1 independent particle systems.  Their particles are
// concatenated (system s owns positions [Sys.p0, Sys.p1) in every particle
// array, and keeps them: sorting is within systems), their tree nodes share
// one level-ordered array (all roots first, root of system s at index s), and
// their sink groups share one group table.  One launch per phase serves all
// systems; a single system is the case S = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Invariant checks compiled only into host-emulation builds of the kernels.
#ifdef HTREE_EMU_CHECKS
#include <cstdio>
#include <cstdlib>
#define HT_CHECK(c)                                                                    \
    do {                                                                               \
        if (!(c)) {                                                                    \
            fprintf(stderr, "HT_CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c);  \
            abort();                                                                   \
        }                                                                              \
    } while (0)
#else
#define HT_CHECK(c) ((void)0)
#endif

namespace htree {

constexpr int kMaxLevel = 21;          // 63-bit keys: 21 levels of 3 bits
// Recorded hard searches (reused on the hard substeps between builds): the
// search radius is widened by kHardSkin R2, and a group of ns sinks starting
// at sorted position b0 keeps up to kListPerSink * ns node ids at
// kListPerSink * b0; a longer list is not kept (the group then walks from
// the root every time).
constexpr double kHardSkin = 0.25;
constexpr uint32_t kListPerSink = 24;
constexpr uint32_t kNoList = 0xffffffffu;
constexpr int kWave = 64;

// Build frame of one system, written by the bounding-box kernels.
struct Frame {
    double lo[3];       // coordinate minimum
    double side;        // root cube side, a power of two >= extent
    double scale;       // 2^21 / side (exact power of two)
    double R2pad2;      // (R2 + slack)^2 for conservative neighbour pruning
    double R2rec2;      // (R2 (1 + kHardSkin) + slack)^2: radius of a recorded hard search
};

// Per-system build parameters (device table).
struct Sys {
    uint32_t p0, p1;    // particle range
    uint32_t c0, c1;    // bounding-box chunk range
    uint32_t n_crit;    // a cell splits while it holds >= n_crit particles
    uint32_t g;         // sink group size (<= 64)
    uint32_t gcell;     // soft groups: chunking cells hold at most gcell * g particles
    uint32_t pad;
    double invth2;      // 1 / theta^2 (+inf for theta = 0)
    double R2;          // hybrid cutoff, 0 in plain mode
    double aerr;        // absolute MAC parameter a_err (0: opening radius l / theta)
    double G;           // gravitational constant (in the absolute MAC)
};

// Per-system force parameters (device table).
struct SysF {
    float G, eps2, R2f, invdR;        // FP32 soft interaction
    double R2sq;                      // exact cutoff test
    double Gd, eps2d, R2d, invdR64;   // FP64 hard interaction
};

// One tree node in level (breadth-first) order; children of a node are
// contiguous.  96 bytes, read as six 16-byte loads by the walks.
struct alignas(16) Node {
    double com[3];      // centre of mass, build frame
    double M;           // mass
    double blo[3];      // lower corner of the cell box, build frame (exact)
    double l;           // cell side
    double rb2;         // squared opening radius (l*l) / theta^2
    uint32_t first;     // first particle (sorted position)
    uint32_t count;     // number of particles
    uint32_t child;     // index of the first child (internal nodes)
    uint32_t meta;      // nchild | level << 8
    uint32_t parent;    // index of the parent (root: itself)
    uint32_t sys;       // system
};
static_assert(sizeof(Node) == 96, "node record layout");

// ---------------------------------------------------------------------------
// wavefront helpers (wave64)
// ---------------------------------------------------------------------------
__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Inclusive scans over the 64 lanes with DPP moves (no LDS round trips):
// shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the row totals by
// the GFX9 row broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2
// and 3).  Lanes a move does not write, or whose source lies outside the
// row, take 0 (the identity of + and of max on unsigned values).  All 64
// lanes must be active.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_u32<0x111, 0xf>(v);
    v += dpp_u32<0x112, 0xf>(v);
    v += dpp_u32<0x114, 0xf>(v);
    v += dpp_u32<0x118, 0xf>(v);
    v += dpp_u32<0x142, 0xa>(v);
    v += dpp_u32<0x143, 0xc>(v);
    return v;
}
__device__ inline uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane(wave_incl_scan(v), 63);
}
__device__ inline uint32_t max_u32(uint32_t a, uint32_t b) { return a > b ? a : b; }
// FP64 minimum / maximum over the 64 lanes, returned in every lane: the same
// DPP pattern on both halves of the value, with +inf / -inf for lanes a
// move does not write.  All 64 lanes must be active.
template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double v, double idle) {
    const uint64_t b = (uint64_t)__double_as_longlong(v), o = (uint64_t)__double_as_longlong(idle);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b,
                                                              CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32),
                                                              (int)(uint32_t)(b >> 32), CTRL,
                                                              ROWS, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline double lane63_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline double wave_min(double v) {
    const double e = INFINITY;
    v = fmin(v, dpp_f64<0x111, 0xf>(v, e));
    v = fmin(v, dpp_f64<0x112, 0xf>(v, e));
    v = fmin(v, dpp_f64<0x114, 0xf>(v, e));
    v = fmin(v, dpp_f64<0x118, 0xf>(v, e));
    v = fmin(v, dpp_f64<0x142, 0xa>(v, e));
    v = fmin(v, dpp_f64<0x143, 0xc>(v, e));
    return lane63_f64(v);
}
__device__ inline double wave_max(double v) {
    const double e = -INFINITY;
    v = fmax(v, dpp_f64<0x111, 0xf>(v, e));
    v = fmax(v, dpp_f64<0x112, 0xf>(v, e));
    v = fmax(v, dpp_f64<0x114, 0xf>(v, e));
    v = fmax(v, dpp_f64<0x118, 0xf>(v, e));
    v = fmax(v, dpp_f64<0x142, 0xa>(v, e));
    v = fmax(v, dpp_f64<0x143, 0xc>(v, e));
    return lane63_f64(v);
}
__device__ inline uint32_t wave_incl_max(uint32_t v) {
    v = max_u32(v, dpp_u32<0x111, 0xf>(v));
    v = max_u32(v, dpp_u32<0x112, 0xf>(v));
    v = max_u32(v, dpp_u32<0x114, 0xf>(v));
    v = max_u32(v, dpp_u32<0x118, 0xf>(v));
    v = max_u32(v, dpp_u32<0x142, 0xa>(v));
    v = max_u32(v, dpp_u32<0x143, 0xc>(v));
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane(wave_incl_max(v), 63);
}

// Sticky device status bits.
enum : uint32_t { kStatusNonFinite = 1u, kStatusOverflow = 2u };

// Radix-sort tile: 256 threads x 8 items (2048 keys; at N = 2^20, 512 tiles
// keep two blocks on each CU through the scatter's barrier-separated rounds).
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

inline int64_t sort_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Workspace slices for the build (device pointers) and the host-side sizes.
struct BuildBufs {
    int64_t n;             // particles over all systems
    int32_t S;             // systems
    int32_t sysbits;       // bits of a system index (0 for S = 1)
    int32_t max_n_crit;    // largest n_crit of the systems
    bool abs_mac;          // some system opens cells by the absolute MAC
    int64_t nchunks;       // bounding-box chunks
    // static tables
    Sys *sys;              // [S]
    SysF *sysf;            // [S]
    uint32_t *sys_of;      // [n] system of each particle position
    uint2 *chunk;          // [nchunks] particle range of each bounding-box chunk
    // particle state, two copies each; cur selects the live copy
    double *x[2];          // [3][n]
    float *v[2];           // [3][n]
    float *m[2];           // [n]
    uint32_t *perm[2];     // [n] sorted position -> caller index
    float *as[2];          // [3][n] soft acceleration (sorted order)
    float *ah[2];          // [3][n] hard acceleration
    uint32_t *wsoft[2];    // [n] cost of each particle's soft group in the last launch
    uint32_t *whard[2];    // [n] and of its hard group (dispatch estimates for new groups)
    int cur;
    double4 *src;          // [n] build-frame position and mass
    uint64_t *key[2];      // [n] sort keys (ping-pong)
    uint32_t *idx[2];      // [n] sort payload
    uint32_t *skey[2];     // [n] system keys for the per-system ordering (S > 1)
    uint64_t *ktmp;        // [n] key scratch for the per-system ordering (S > 1)
    uint32_t *hist;        // radix histograms (+ scan partials)
    double *bbox_part;     // [nchunks][6]
    Frame *frame;          // [S]
    uint32_t *status;      // sticky status word
    // topology
    int8_t *cpl;           // [n] common-prefix level with the previous key
    int8_t *leaflev;       // [n] leaf level of each particle
    uint32_t *nstart;      // [n+1] nodes starting at each position, scanned
    uint32_t *scan_part;   // scan partials
    uint32_t *nn;          // [4] device node count in nn[0]; nn[2] work items of the b_max pass
    uint32_t *pre_key;     // [nnmax] (level, system) key of each pre-order node
    uint32_t *pre_val;     // [nnmax] pre-order index
    uint32_t *lvl_key2;    // [nnmax] partitioned keys
    uint32_t *bfs2pre;     // [nnmax]
    uint32_t *pre2bfs;     // [nnmax]
    uint32_t *pre_first;   // [nnmax]
    uint32_t *pre_count;   // [nnmax]
    uint32_t *ptmp_k, *ptmp_v;  // [nnmax] partition scratch
    Node *node;            // [nnmax] level order
    double *S3;            // [3][nnmax] first mass moments
    double4 *xm;           // [n] key-order master positions and masses (x, y, z, m) in one
                           // record per particle, for the hard kernel's gathers; written by
                           // the gather of each build and by every drift
    double *aabb;          // [nnmax][8] node boxes in master coordinates: lo x, y, z, -, hi x, y, z, -
    double *cbox;          // boxes of aligned 32, 32^2, 32^3-particle chunks (refit)
    uint32_t *lstart;      // [kMaxLevel + 2] first node of each level
    int64_t nnmax;
    // sink groups
    uint32_t *gstart;      // [n+1] soft group start positions (ng + 1 used)
    uint32_t *ng;          // device soft group count
    uint32_t *hgstart;     // [n+1] hard group start positions (nhg + 1 used)
    uint32_t *nhg;         // device hard group count
    // hard-group dispatch order (measured costs, heaviest first)
    uint32_t *hcost;       // [2n] cost of each hard group in the last launch; sort scratch
    uint32_t *hkey;        // [2n] sort keys (descending cost buckets)
    uint32_t *hval;        // [2n] group indices before the sort
    uint32_t *horder;      // [n] dispatch position -> hard group
    double *B2;            // [nnmax] sum m |COM - u|^2 per node (absolute MAC only)
    unsigned long long *bmax;  // [nnmax] bits of max |COM - u|^2 per node (absolute MAC only)
    uint32_t *bitems;      // [nnmax + 1] work items of the b_max pass (absolute MAC only)
    uint32_t *hlist;       // [kListPerSink * n] recorded hard search lists (node ids)
    uint32_t *hlen;        // [n] their lengths per hard group, or kNoList
    uint32_t *sorder;      // [2n] dispatch position -> soft group (first ng entries)
    uint32_t *ndisp;       // device count of the dispatch sort (ng + nhg)
};

// Host launch wrappers (build.hip).
void launch_bbox_keys(const BuildBufs &B, hipStream_t s);
void launch_sort(BuildBufs &B, hipStream_t s);
void launch_gather(BuildBufs &B, bool keep_acc, hipStream_t s);
void launch_topology(BuildBufs &B, bool moments, hipStream_t s);
void launch_levels(BuildBufs &B, bool moments, hipStream_t s);
void launch_refit(BuildBufs &B, hipStream_t s);
void refit_sizes(int64_t n, int64_t *m1, int64_t *m2, int64_t *m3);
void launch_groups(BuildBufs &B, hipStream_t s);
void launch_hard_order(BuildBufs &B, hipStream_t s);
void launch_dispatch_orders(BuildBufs &B, hipStream_t s);
void launch_sys_of(BuildBufs &B, hipStream_t s);
size_t scan_partials(int64_t n);
void launch_scan_u32(uint32_t *data, int64_t n, uint32_t *part, uint32_t *total, hipStream_t s);

// Interaction tallies (soft interactions, hard candidates, hard pairs) are
// added by every sink group.  Device-scope atomics of many workgroups on one
// address serialize, so the counters live in kTallySlots slots, one 128-byte
// line each, picked by workgroup index; launch_tally_fold sums the slots into
// four totals.
constexpr int kTallySlots = 32;
constexpr int kTallyStride = 16;
void launch_tally_fold(const unsigned long long *slots, unsigned long long *sum, hipStream_t s);

// Force kernels (force.hip).
struct ForceArgs {
    const Node *node;
    const uint32_t *gstart;   // group k is sorted positions [gstart[k], gstart[k+1])
    const uint32_t *ng;       // device group count
    const uint32_t *sys_of;   // [n]
    const SysF *sysf;         // [S]
    const double4 *src;       // sorted build-frame positions and masses
    const double4 *xm;        // [n] key-order master positions and masses (hard kernel)
    const double *aabb;       // [nnmax][8] node boxes, master coordinates (lo xyz, -, hi xyz, -)
    int64_t nnmax;
    const Frame *frame;       // [S]
    const uint32_t *order;    // null, or dispatch position -> group (a permutation)
    uint32_t *cost;           // null, or [ng] per-group work measure written by the hard kernel
    uint32_t *hlist;          // hard kernel: recorded search lists (see kListPerSink)
    uint32_t *hlen;           // hard kernel: their lengths per group
    int32_t hmode;            // hard kernel: 0 walk from the root, 1 record, 2 replay
    uint32_t *wsoft;          // null, or [n]: each soft group writes its work measure to its sinks
    int64_t n;
    float *acc;               // [3][n] sorted order output
    float *pot;               // [n] or null
    int32_t *ngb;             // [n] or null
    uint32_t *gcount;         // [3][n] list sizes per group (first ng used) or null
    unsigned long long *tally;  // [kTallySlots][kTallyStride] interaction tally slots
    uint32_t *status;
};
void launch_soft(const ForceArgs &A, bool hybrid, bool pot, int precision, bool min_sinks,
                 int n_wg, hipStream_t s);
void launch_hard(const ForceArgs &A, int n_wg, hipStream_t s);

// Integrator and layout kernels (integrate.hip).
void launch_kick_drift(double *x, double4 *xm, const float *m, float *v, const float *a1, float c1,
                       const float *a2, float c2, double dt_drift, int64_t n, hipStream_t s);
void launch_scatter3(const float *src_sorted, const uint32_t *perm, float *dst, int64_t n,
                     hipStream_t s);
void launch_scatter1f(const float *src_sorted, const uint32_t *perm, float *dst, int64_t n,
                      hipStream_t s);
void launch_scatter1i(const int32_t *src_sorted, const uint32_t *perm, int32_t *dst, int64_t n,
                      hipStream_t s);
void launch_gather3(const float *src_caller, const uint32_t *perm, float *dst_sorted, int64_t n,
                    hipStream_t s);
void launch_scatter_x(const double *x_sorted, const uint32_t *perm, double *dst, int64_t n,
                      hipStream_t s);
void launch_set_state(const double *x, int64_t ldx, const float *v, const float *m, double *xs,
                      float *vs, float *ms, uint32_t *perm, int64_t n, hipStream_t s);
void launch_add3(const float *a, const float *b, float *out, int64_t n, hipStream_t s);
void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);

}  // namespace htree
