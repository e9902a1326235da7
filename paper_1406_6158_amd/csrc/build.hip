// build.hip -- octree construction on the GPU (section III.A.1 of the paper,
// redesigned for gfx950) for S independent systems at once: bounding boxes,
// 63-bit Morton keys, stable LSD radix sort within each system, state
// permutation, topology from the sorted keys, level-by-level moments, sink
// groups.
//
// Topology without recursion.  The paper splits the sorted array recursively
// by 3-bit key digits while a cell holds >= n_crit particles.  The same tree
// is obtained in parallel: with c_i the number of leading 3-bit digits that
// key i shares with key i-1 (-1 at a system's first particle), and D_i the
// largest number of digits shared by the two ends of any window of n_crit
// consecutive keys of the same system containing i, the cell of level l
// around particle i holds >= n_crit particles iff l <= D_i.  Hence particle
// i's leaf is at level L_i = min(D_i + 1, 21) (0 if the system has fewer than
// n_crit particles), and the nodes that begin at sorted position i are the
// cells of levels c_i + 1 .. L_i.  Enumerating them by position gives the
// depth-first (pre-order) node sequence; a stable partition by (level,
// system) gives level order, in which the children of a node are contiguous
// and the root of system s is node s.
#include "htree_dev.h"

#include <math.h>

namespace htree {

// ---------------------------------------------------------------------------
// block scan helper
// ---------------------------------------------------------------------------
// Exclusive scan across a block of NT threads; returns the prefix and writes
// the block total.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t t = lane < NT / 64 ? sh[lane] : 0u;
        uint32_t ti = wave_incl_scan(t);
        if (lane < NT / 64) sh[lane] = ti - t;
        if (lane == NT / 64 - 1) sh[NT / 64] = ti;
    }
    __syncthreads();
    uint32_t r = inc - v + sh[w];
    total = sh[NT / 64];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// exclusive scan of a u32 array (in place), with the grand total
// ---------------------------------------------------------------------------
constexpr int kScanNT = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanNT * kScanItems;

size_t scan_partials(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint32_t *data, int64_t n,
                                                         uint32_t *part) {
    __shared__ uint32_t sh[kScanNT / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = base + k * kScanNT + threadIdx.x;
        if (i < n) s += data[i];
    }
    uint32_t tot;
    block_excl_scan<kScanNT>(s, sh, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t *part, int64_t np,
                                                        uint32_t *total) {
    __shared__ uint32_t sh[1024 / 64 + 1];
    uint32_t carry = 0;
    for (int64_t c = 0; c < np; c += 1024) {
        int64_t i = c + threadIdx.x;
        uint32_t v = i < np ? part[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan<1024>(v, sh, tot);
        if (i < np) part[i] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// SELF: the block adds up the block sums before its own (part[0, blockIdx.x))
// instead of reading their prefix from k_scan_partials, and the last block
// writes the grand total; used while the blocks are few.
template <bool SELF>
__global__ __launch_bounds__(kScanNT) void k_scan_down(uint32_t *data, int64_t n,
                                                       const uint32_t *part, uint32_t *total) {
    __shared__ uint32_t sh[kScanNT / 64 + 1];
    int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint32_t before = 0;
    if (SELF) {
        uint32_t p = 0;
        for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kScanNT) p += part[j];
        block_excl_scan<kScanNT>(p, sh, before);
    } else {
        before = part[blockIdx.x];
    }
    // each thread owns kScanItems consecutive elements
    uint32_t v[kScanItems];
    uint32_t s = 0;
    int64_t t0 = base + (int64_t)threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = t0 + k;
        v[k] = i < n ? data[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<kScanNT>(s, sh, tot) + before;
    for (int k = 0; k < kScanItems; k++) {
        int64_t i = t0 + k;
        if (i < n) data[i] = ex;
        ex += v[k];
    }
    if (SELF && total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = before + tot;
}

constexpr int64_t kScanSelfMax = 4096;   // blocks up to which k_scan_down sums the prefix itself

void launch_scan_u32(uint32_t *data, int64_t n, uint32_t *part, uint32_t *total, hipStream_t s) {
    int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanNT), 0, s, data, n, part);
    if (nb <= kScanSelfMax) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3((unsigned)nb), dim3(kScanNT), 0, s, data, n,
                           part, total);
    } else {
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, part, nb, total);
        hipLaunchKernelGGL(k_scan_down<false>, dim3((unsigned)nb), dim3(kScanNT), 0, s, data, n,
                           part, nullptr);
    }
}

// ---------------------------------------------------------------------------
// static system table: system of each particle position
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sys_of(const Sys *sys, int S, int64_t n,
                                                uint32_t *sys_of) {
    // one thread per particle: the last system whose range starts at or before it
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys[mid].p0 <= (uint32_t)i) lo = mid; else hi = mid - 1;
    }
    sys_of[i] = (uint32_t)lo;
}

void launch_sys_of(BuildBufs &B, hipStream_t s) {
    hipLaunchKernelGGL(k_sys_of, dim3((unsigned)((B.n + 255) / 256)), dim3(256), 0, s, B.sys,
                       B.S, B.n, B.sys_of);
}

// ---------------------------------------------------------------------------
// bounding boxes, frames and keys
// ---------------------------------------------------------------------------
constexpr int kBoxNT = 256;

// One block per chunk of one system's particles.
__global__ __launch_bounds__(kBoxNT) void k_bbox(const double *x, int64_t n, const uint2 *chunk,
                                                 double *part, uint32_t *status) {
    __shared__ double sh[kBoxNT / 64][6];
    const uint2 c = chunk[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (uint32_t i = c.x + threadIdx.x; i < c.y; i += kBoxNT) {
        for (int a = 0; a < 3; a++) {
            double v = x[a * n + i];
            bad |= !isfinite(v);
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    }
    if (bad) atomicOr(status, kStatusNonFinite);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int a = 0; a < 3; a++) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane == 0)
        for (int a = 0; a < 3; a++) { sh[w][a] = lo[a]; sh[w][3 + a] = hi[a]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBoxNT / 64; k++)
            for (int a = 0; a < 3; a++) {
                sh[0][a] = fmin(sh[0][a], sh[k][a]);
                sh[0][3 + a] = fmax(sh[0][3 + a], sh[k][3 + a]);
            }
        for (int a = 0; a < 6; a++) part[(int64_t)blockIdx.x * 6 + a] = sh[0][a];
    }
}

// One block per system: reduce its chunks, then fix the build frame.
__global__ __launch_bounds__(kBoxNT) void k_frame(const double *part, const Sys *sys,
                                                  Frame *frames) {
    __shared__ double sh[kBoxNT / 64][6];
    const Sys S = sys[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = S.c0 + threadIdx.x; b < S.c1; b += kBoxNT)
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], part[(int64_t)b * 6 + a]);
            hi[a] = fmax(hi[a], part[(int64_t)b * 6 + 3 + a]);
        }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int a = 0; a < 3; a++) {
        lo[a] = wave_min(lo[a]);
        hi[a] = wave_max(hi[a]);
    }
    if (lane == 0)
        for (int a = 0; a < 3; a++) { sh[w][a] = lo[a]; sh[w][3 + a] = hi[a]; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int a = 0; a < 3; a++) {
        lo[a] = sh[0][a];
        hi[a] = sh[0][3 + a];
        for (int k = 1; k < kBoxNT / 64; k++) {
            lo[a] = fmin(lo[a], sh[k][a]);
            hi[a] = fmax(hi[a], sh[k][3 + a]);
        }
    }
    // extent of the build frame u = x - lo: rounding is monotone, so the
    // largest rounded difference is the rounded difference of the extremes
    double ext = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = hi[a] - lo[a];
        if (e > ext) ext = e;
    }
    double side;
    if (!(ext > 0.0)) {
        side = 1.0;
    } else {
        int e;
        double f = frexp(ext, &e);
        side = (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
    }
    Frame &F = frames[blockIdx.x];
    for (int a = 0; a < 3; a++) F.lo[a] = lo[a];
    F.side = side;
    F.scale = ldexp(1.0, kMaxLevel) / side;
    // slack covers the rounding of build-frame differences against FP64 x
    double R2p = S.R2 + ldexp(side, -40);
    F.R2pad2 = R2p * R2p;
    double R2r = S.R2 * (1.0 + kHardSkin) + ldexp(side, -40);
    F.R2rec2 = R2r * R2r;
}

__device__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__global__ __launch_bounds__(256) void k_keys(const double *x, int64_t n, const uint32_t *sys_of,
                                              const Frame *frames, uint64_t *key, uint32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Frame &F = frames[sys_of[i]];
    const double scale = F.scale;
    const uint32_t qmax = (1u << kMaxLevel) - 1u;
    uint32_t q[3];
    for (int a = 0; a < 3; a++) {
        double u = x[a * n + i] - F.lo[a];
        double s = floor(u * scale);
        q[a] = (s >= (double)qmax) ? qmax : (uint32_t)s;
    }
    key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[i] = (uint32_t)i;
}

void launch_bbox_keys(const BuildBufs &B, hipStream_t s) {
    int64_t n = B.n;
    const double *x = B.x[B.cur];
    hipLaunchKernelGGL(k_bbox, dim3((unsigned)B.nchunks), dim3(kBoxNT), 0, s, x, n, B.chunk,
                       B.bbox_part, B.status);
    hipLaunchKernelGGL(k_frame, dim3((unsigned)B.S), dim3(kBoxNT), 0, s, B.bbox_part, B.sys,
                       B.frame);
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, B.sys_of,
                       B.frame, B.key[0], B.idx[0]);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *key, int64_t nmax,
                                                             const uint32_t *count_dev, int shift,
                                                             uint32_t *hist, int64_t nb) {
    __shared__ uint32_t cnt[256];
    const int tid = threadIdx.x;
    const int64_t n = count_dev ? (int64_t)*count_dev : nmax;
    cnt[tid] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; r++) {
        int64_t i = base + r * kSortThreads + tid;
        if (i < n) atomicAdd(&cnt[(uint32_t)(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nb + blockIdx.x] = cnt[tid];
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const K *key, const uint32_t *val, int64_t nmax, const uint32_t *count_dev, int shift,
    const uint32_t *hist, int64_t nb, K *key_out, uint32_t *val_out) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int tid = threadIdx.x, w = tid >> 6;
    const int64_t n = count_dev ? (int64_t)*count_dev : nmax;
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    if (tile0 >= n) return;
    run[tid] = 0;
    base[tid] = hist[(int64_t)tid * nb + blockIdx.x];
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kSortItems; r++) {
        int64_t i = tile0 + r * kSortThreads + tid;
        bool valid = i < n;
        K k = valid ? key[i] : (K)0;
        uint32_t v = valid ? val[i] : 0u;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        for (int j = 0; j < kSortThreads / 64; j++) wcnt[j][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int j = 0; j < w; j++) pre += wcnt[j][d];
            uint32_t pos = base[d] + run[d] + pre + rank;
            key_out[pos] = k;
            val_out[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int j = 0; j < kSortThreads / 64; j++) add += wcnt[j][tid];
        run[tid] += add;
        __syncthreads();
    }
}

template <typename K>
static void radix_pass(const K *kin, const uint32_t *vin, K *kout, uint32_t *vout,
                       uint32_t *hist, uint32_t *part, const uint32_t *count_dev, int64_t nmax,
                       int shift, hipStream_t s) {
    int64_t nb = sort_blocks(nmax);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, nmax,
                       count_dev, shift, hist, nb);
    launch_scan_u32(hist, 256 * nb, part, nullptr, s);
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, vin,
                       nmax, count_dev, shift, hist, nb, kout, vout);
}

// system of each entry of the Morton-ordered sequence, and its position
__global__ __launch_bounds__(256) void k_sys_keys(const uint32_t *idx, const uint32_t *sys_of,
                                                  int64_t n, uint32_t *skey, uint32_t *pos) {
    int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    skey[p] = sys_of[idx[p]];
    pos[p] = (uint32_t)p;
}

// apply the per-system reordering to the Morton-ordered keys and payload
__global__ __launch_bounds__(256) void k_apply_order(const uint32_t *pos, const uint64_t *key_in,
                                                     const uint32_t *idx_in, int64_t n,
                                                     uint64_t *key_out, uint32_t *idx_out) {
    int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    uint32_t p = pos[q];
    key_out[q] = key_in[p];
    idx_out[q] = idx_in[p];
}

void launch_sort(BuildBufs &B, hipStream_t s) {
    // keys are 63-bit: eight passes, the result lands back in buffer 0
    for (int pass = 0; pass < 8; pass++) {
        int a = pass & 1, b = a ^ 1;
        radix_pass<uint64_t>(B.key[a], B.idx[a], B.key[b], B.idx[b], B.hist, B.scan_part, nullptr,
                             B.n, 8 * pass, s);
    }
    if (B.S > 1) {
        // stable passes on the system index keep each system's key order and
        // put every system back on its own particle range
        const int64_t n = B.n;
        unsigned gb = (unsigned)((n + 255) / 256);
        uint32_t *pos[2] = {B.idx[1], (uint32_t *)B.key[1]};
        hipLaunchKernelGGL(k_sys_keys, dim3(gb), dim3(256), 0, s, B.idx[0], B.sys_of, n,
                           B.skey[0], pos[0]);
        int cur = 0;
        for (int sh = 0; sh < B.sysbits; sh += 8) {
            radix_pass<uint32_t>(B.skey[cur], pos[cur], B.skey[cur ^ 1], pos[cur ^ 1], B.hist,
                                 B.scan_part, nullptr, n, sh, s);
            cur ^= 1;
        }
        // Morton keys and payload in final order go to spare buffers (ktmp
        // holds n 64-bit keys; pos[cur ^ 1] is free), then back to buffer 0
        hipLaunchKernelGGL(k_apply_order, dim3(gb), dim3(256), 0, s, pos[cur], B.key[0], B.idx[0],
                           n, B.ktmp, pos[cur ^ 1]);
        (void)hipMemcpyAsync(B.key[0], B.ktmp, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(B.idx[0], pos[cur ^ 1], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice,
                             s);
    }
}

// Dispatch order of the hard groups for the next launches over the same
// groups: heaviest first (by the costs the last launch measured), so that the
// expensive groups of dense regions do not start late and leave a tail of a
// few long workgroups.  Costs are bucketed at a quarter octave; the stable
// sort keeps key order inside a bucket.
// Quarter-octave bucket of a cost (0 .. 127).
__device__ inline uint32_t cost_bucket(uint32_t c) {
    if (c == 0) return 0;
    const uint32_t e = 31u - (uint32_t)__builtin_clz(c);
    const uint32_t f = e >= 2 ? (c >> (e - 2)) & 3u : (c << (2 - e)) & 3u;
    return 4 * e + f;
}

__global__ __launch_bounds__(256) void k_hard_order_keys(const uint32_t *cost, const uint32_t *nhg,
                                                         uint32_t *key, uint32_t *val) {
    const uint32_t g = blockIdx.x * 256 + threadIdx.x;
    if (g >= *nhg) return;
    key[g] = 255u - cost_bucket(cost[g]);
    val[g] = g;
}

// Keys of both kinds of new groups for one sort: soft group g at entry g with
// key 127 - bucket, hard group h at entry ng + h with key 255 - bucket, so
// the sorted values hold the soft order in [0, ng) and the hard order in
// [ng, ng + nhg).  A group's estimate is the mean over its sinks of the cost
// of the group each sink belonged to in the last launch (particles move
// little between builds); before any launch all estimates are 0 (key order).
// One wavefront per group, four per block.
__global__ __launch_bounds__(256) void k_dispatch_keys(const uint32_t *gstart, const uint32_t *ngp,
                                                       const uint32_t *ws, const uint32_t *hgstart,
                                                       const uint32_t *nhgp, const uint32_t *wh,
                                                       uint32_t *key, uint32_t *val,
                                                       uint32_t *total) {
    const uint32_t ng = *ngp, nhg = *nhgp;
    const int lane = __lane_id();
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = ng + nhg;
    for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < ng + nhg; g += gridDim.x * 4) {
        const bool soft = g < ng;
        const uint32_t k = soft ? g : g - ng;
        const uint32_t *st = soft ? gstart : hgstart;
        const uint32_t *w = soft ? ws : wh;
        const uint32_t b0 = st[k], ns = st[k + 1] - b0;
        uint64_t sum = lane < (int)ns ? w[b0 + lane] : 0u;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
        if (lane == 0) {
            const uint64_t mean = sum / ns;
            const uint32_t b = cost_bucket(mean > 0xffffffffull ? 0xffffffffu : (uint32_t)mean);
            key[g] = (soft ? 127u : 255u) - b;
            val[g] = k;
        }
    }
}

__global__ __launch_bounds__(256) void k_order_tail(const uint32_t *sorted, const uint32_t *ngp,
                                                    const uint32_t *nhgp, uint32_t *horder) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < *nhgp) horder[k] = sorted[*ngp + k];
}

// The measured cost of each hard group, written to its sinks (carried to the
// next build's groups by the gather).  One wavefront per group.
__global__ __launch_bounds__(256) void k_spread_cost(const uint32_t *hgstart, const uint32_t *nhgp,
                                                     const uint32_t *cost, uint32_t *wh) {
    const uint32_t nhg = *nhgp;
    const int lane = __lane_id();
    for (uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6); g < nhg; g += gridDim.x * 4) {
        const uint32_t b0 = hgstart[g], ns = hgstart[g + 1] - b0;
        if (lane < (int)ns) wh[b0 + lane] = cost[g];
    }
}

static unsigned wave_grid(int64_t n) { return (unsigned)((n + 3) / 4 < 2048 ? (n + 3) / 4 : 2048); }

// Dispatch orders of the new soft and hard groups from the carried costs.
void launch_dispatch_orders(BuildBufs &B, hipStream_t s) {
    const int64_t n = B.n;
    hipLaunchKernelGGL(k_dispatch_keys, dim3(wave_grid(2 * n)), dim3(256), 0, s, B.gstart, B.ng,
                       B.wsoft[B.cur], B.hgstart, B.nhg, B.whard[B.cur], B.hkey, B.hval, B.ndisp);
    radix_pass<uint32_t>(B.hkey, B.hval, B.hcost, B.sorder, B.hist, B.scan_part, B.ndisp, 2 * n, 0,
                         s);
    hipLaunchKernelGGL(k_order_tail, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B.sorder,
                       B.ng, B.nhg, B.horder);
}

// After the first launch over new hard groups: their measured costs go to
// their sinks, and order the later launches.
void launch_hard_order(BuildBufs &B, hipStream_t s) {
    const int64_t n = B.n;
    hipLaunchKernelGGL(k_spread_cost, dim3(wave_grid(n)), dim3(256), 0, s, B.hgstart, B.nhg,
                       B.hcost, B.whard[B.cur]);
    hipLaunchKernelGGL(k_hard_order_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       B.hcost, B.nhg, B.hkey, B.hval);
    radix_pass<uint32_t>(B.hkey, B.hval, B.hcost, B.horder, B.hist, B.scan_part, B.nhg, n, 0, s);
}

// ---------------------------------------------------------------------------
// permutation of the particle state into key order
// ---------------------------------------------------------------------------
// The dispatcher deals workgroups to the 8 XCDs round-robin (XCD = blockIdx %
// 8), each XCD with its own L2.  With a grid of 8 * per blocks, block b takes
// part (b % 8) * per + b / 8 (a bijection onto [0, 8 * per)), so each XCD
// works through one contiguous eighth of the parts.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_part(uint32_t b, uint32_t grid) {
    const uint32_t per = grid / kXcds;
    return (b % kXcds) * per + b / kXcds;
}
inline unsigned xcd_grid(int64_t parts) {
    const int64_t per = (parts + kXcds - 1) / kXcds;
    return (unsigned)(kXcds * (per > 0 ? per : 1));
}

// Between two builds particles move by little in key order, so the rows a
// block gathers lie in a window around its own positions that the
// neighbouring blocks read too: the blocks run in XCD-contiguous order so
// that those rows are fetched into one L2 rather than into all eight.
template <bool ACC>
__global__ __launch_bounds__(256) void k_gather(
    const uint32_t *idx, int64_t n, const uint32_t *sys_of, const Frame *frames, const double *x0,
    const float *v0, const float *m0, const uint32_t *p0, const float *as0, const float *ah0,
    const uint32_t *wc0, const uint32_t *wh0, double *x1, float *v1, float *m1, uint32_t *p1,
    float *as1, float *ah1, uint32_t *wc1, uint32_t *wh1, double4 *src, double4 *xm) {
    int64_t p = (int64_t)xcd_part(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (p >= n) return;
    uint32_t o = idx[p];
    const Frame &F = frames[sys_of[p]];
    double xx[3];
    for (int a = 0; a < 3; a++) {
        xx[a] = x0[a * n + o];
        x1[a * n + p] = xx[a];
        v1[a * n + p] = v0[a * n + o];
        if (ACC) {
            as1[a * n + p] = as0[a * n + o];
            ah1[a * n + p] = ah0[a * n + o];
        }
    }
    float mm = m0[o];
    m1[p] = mm;
    p1[p] = p0[o];
    wc1[p] = wc0[o];
    wh1[p] = wh0[o];
    src[p] = make_double4(xx[0] - F.lo[0], xx[1] - F.lo[1], xx[2] - F.lo[2], (double)mm);
    xm[p] = make_double4(xx[0], xx[1], xx[2], (double)mm);
}

// Permutes the state into the new key order.  The kept accelerations follow
// only if keep_acc (callers that recompute both forces next skip them).
void launch_gather(BuildBufs &B, bool keep_acc, hipStream_t s) {
    int c = B.cur, d = c ^ 1;
    int64_t n = B.n;
    const dim3 grid(xcd_grid((n + 255) / 256));
    if (keep_acc)
        hipLaunchKernelGGL(k_gather<true>, grid, dim3(256), 0, s, B.idx[0], n, B.sys_of, B.frame,
                           B.x[c], B.v[c], B.m[c], B.perm[c], B.as[c], B.ah[c], B.wsoft[c],
                           B.whard[c], B.x[d], B.v[d], B.m[d], B.perm[d], B.as[d], B.ah[d],
                           B.wsoft[d], B.whard[d], B.src, B.xm);
    else
        hipLaunchKernelGGL(k_gather<false>, grid, dim3(256), 0, s, B.idx[0], n, B.sys_of,
                           B.frame, B.x[c], B.v[c], B.m[c], B.perm[c], B.as[c], B.ah[c],
                           B.wsoft[c], B.whard[c], B.x[d], B.v[d], B.m[d], B.perm[d], B.as[d],
                           B.ah[d], B.wsoft[d], B.whard[d], B.src, B.xm);
    B.cur = d;
}

// ---------------------------------------------------------------------------
// topology
// ---------------------------------------------------------------------------
// number of leading 3-bit digits two 63-bit keys share (21 if equal)
__device__ inline int common_levels(uint64_t a, uint64_t b) {
    uint64_t d = a ^ b;
    if (d == 0) return kMaxLevel;
    return (__clzll((long long)d) - 1) / 3;
}

__global__ __launch_bounds__(256) void k_cpl(const uint64_t *key, int64_t n,
                                             const uint32_t *sys_of, const Sys *sys, int8_t *cpl,
                                             int8_t *dwin) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Sys S = sys[sys_of[i]];
    uint64_t k = key[i];
    cpl[i] = (int8_t)((uint32_t)i == S.p0 ? -1 : common_levels(key[i - 1], k));
    // window of n_crit keys starting at i, inside the system
    int64_t j = i + (int64_t)S.n_crit - 1;
    dwin[i] = (int8_t)(j < (int64_t)S.p1 ? common_levels(k, key[j]) : -1);
}

__global__ __launch_bounds__(256) void k_leaflev(const int8_t *cpl, const int8_t *dwin, int64_t n,
                                                 const uint32_t *sys_of, const Sys *sys,
                                                 int8_t *leaflev, uint32_t *nstart) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const Sys S = sys[sys_of[i]];
    const int64_t p0 = S.p0;
    int D = -1;
    int64_t s0 = i - (int64_t)S.n_crit + 1;
    if (s0 < p0) s0 = p0;
    for (int64_t s = s0; s <= i; s++) {
        int d = dwin[s];   // -1 where the window runs past the system's end
        if (d > D) D = d;
    }
    int L = D < 0 ? 0 : (D + 1 < kMaxLevel ? D + 1 : kMaxLevel);
    leaflev[i] = (int8_t)L;
    int c = cpl[i];
    nstart[i] = (uint32_t)(L > c ? L - c : 0);
    if (i == n - 1) nstart[n] = 0u;   // the scan's total must not see stale data
}

// end of the level-lev cell that starts at sorted position i (within [i, p1))
__device__ inline uint32_t cell_end(const uint64_t *key, int64_t p1, int64_t i, int lev) {
    int sh = 3 * (kMaxLevel - lev);
    uint64_t P = key[i] >> sh;
    // gallop then bisect for the first j > i with a different prefix
    int64_t lo = i, step = 1, hi;
    for (;;) {
        hi = lo + step;
        if (hi >= p1) { hi = p1; break; }
        if ((key[hi] >> sh) != P) break;
        lo = hi;
        step <<= 1;
    }
    // key[lo] has prefix P; key[hi] differs (or hi == p1)
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if ((key[mid] >> sh) == P) lo = mid; else hi = mid;
    }
    return (uint32_t)hi;
}

__global__ __launch_bounds__(256) void k_emit_pre(const int8_t *cpl, const uint32_t *nstart,
                                                  int64_t n, const uint32_t *sys_of, int sysbits,
                                                  uint32_t *pre_key, uint32_t *pre_val,
                                                  uint32_t *pre_first) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t p0 = nstart[i], p1 = nstart[i + 1];
    const uint32_t s = sys_of[i];
    int lev = cpl[i] + 1;
    for (uint32_t p = p0; p < p1; p++, lev++) {
        pre_key[p] = ((uint32_t)lev << sysbits) | s;
        pre_val[p] = p;
        pre_first[p] = (uint32_t)i;
    }
}

// Particle count of every pre-order node: the end of its cell in key order
// (one thread per node, so the nodes that share a first particle -- the root
// and its first descendants -- are searched side by side, not one after
// another by that particle's thread).  Blocks stride over the nodes.
__global__ __launch_bounds__(256) void k_node_count(const uint64_t *key, const uint32_t *pre_key,
                                                    const uint32_t *pre_first, const uint32_t *nn,
                                                    const Sys *sys, int sysbits,
                                                    uint32_t *pre_count) {
    const uint32_t n_nodes = *nn;
    for (uint32_t p = blockIdx.x * 256 + threadIdx.x; p < n_nodes; p += gridDim.x * 256) {
        const uint32_t k = pre_key[p];
        const int lev = (int)(k >> sysbits);
        const uint32_t s = k & ((1u << sysbits) - 1u);
        const uint32_t i = pre_first[p];
        pre_count[p] = cell_end(key, sys[s].p1, i, lev) - i;
    }
}

__global__ __launch_bounds__(256) void k_pre2bfs(const uint32_t *bfs2pre, const uint32_t *nn,
                                                 uint32_t *pre2bfs) {
    uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= *nn) return;
    pre2bfs[bfs2pre[b]] = b;
}

__global__ __launch_bounds__(256) void k_fill_nodes(
    const uint64_t *key, const int8_t *leaflev, const uint32_t *nstart, const uint32_t *bfs2pre,
    const uint32_t *pre2bfs, const uint32_t *lkey, const uint32_t *pre_first,
    const uint32_t *pre_count, const uint32_t *nn, const Frame *frames, const Sys *sys,
    int sysbits, Node *node) {
    uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= *nn) return;
    uint32_t p = bfs2pre[b];
    const uint32_t k = lkey[b];
    const int lev = (int)(k >> sysbits);
    const uint32_t s = k & ((1u << sysbits) - 1u);
    uint32_t first = pre_first[p], count = pre_count[p];
    bool internal = lev < leaflev[first];
    uint32_t child = 0, nch = 0;
    if (internal) {
        child = pre2bfs[p + 1];
        uint32_t c = p + 1, end = first + count;
        for (;;) {
            nch++;
            uint32_t e = pre_first[c] + pre_count[c];
            if (e >= end) break;
            c = nstart[e];
        }
        for (uint32_t j = 0; j < nch; j++) node[child + j].parent = b;
    }
    if (lev == 0) node[b].parent = b;
    const Frame &F = frames[s];
    double l = ldexp(F.side, -lev);
    uint64_t k0 = key[first];
    Node &N = node[b];
    N.first = first;
    N.count = count;
    N.child = child;
    N.meta = nch | ((uint32_t)lev << 8);
    N.sys = s;
    N.l = l;
    N.rb2 = (l * l) * sys[s].invth2;
    for (int a = 0; a < 3; a++) {
        uint32_t q = compact3(k0 >> (2 - a));
        N.blo[a] = (double)(q >> (kMaxLevel - lev)) * l;
    }
}

// Start of each level in the level-ordered node array (levels are contiguous
// and every level from 0 to the deepest one is present); entries past the
// deepest level are set to the node count.  Each entry has a single writer:
// the first node of its level, or the last node for the levels beyond.
__global__ __launch_bounds__(256) void k_level_starts(const uint32_t *lkey, int sysbits,
                                                      const uint32_t *nn_dev, uint32_t *lstart) {
    uint32_t b = blockIdx.x * 256 + threadIdx.x;
    uint32_t nn = *nn_dev;
    if (b >= nn) return;
    uint32_t l = lkey[b] >> sysbits;
    if (b == 0 || (lkey[b - 1] >> sysbits) != l) lstart[l] = b;
    if (b == nn - 1)
        for (uint32_t m = l + 1; m <= (uint32_t)kMaxLevel + 1; m++) lstart[m] = nn;
}

// Node box record b: 8 doubles (lo x, y, z, unused, hi x, y, z, unused), one
// 64-byte line half, so a walk reads a node's box with two 32-byte loads.
__device__ inline void store_box(double *aabb, uint32_t b, const double *lo, const double *hi) {
    double4 *r = (double4 *)aabb + 2 * (int64_t)b;
    r[0] = make_double4(lo[0], lo[1], lo[2], 0.0);
    r[1] = make_double4(hi[0], hi[1], hi[2], 0.0);
}

// |p - q|^2 as fma(dz, dz, fma(dy, dy, dx * dx)) with d = p - q.
__device__ inline double sqdist(const double *p, double qx, double qy, double qz) {
    const double dx = p[0] - qx, dy = p[1] - qy, dz = p[2] - qz;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// One level of the bottom-up pass, deepest level first.  Every node gets the
// box of its particles' master positions (exact minima and maxima: a leaf
// over its particles, an internal node over its children's boxes).  With
// MOM, also the moments: a leaf sums its particles in sorted order (M += m,
// S = fma(m, u, S)); an internal node sums its children's M and S in octant
// order; COM = S / M.  With MAC (absolute MAC, section II.B eq. 6), also
// B2 = sum m |COM - u|^2: a leaf over its particles in sorted order
// (B2 = fma(m, |COM - u|^2, B2)), an internal node over its children in
// octant order (B2 += fma(M_c, |COM - COM_c|^2, B2_c), the parallel-axis
// identity).
template <bool MOM, bool MAC>
__global__ __launch_bounds__(256) void k_level_pass(Node *node, const double4 *src, const double *x,
                                                    int64_t n, double *S3, double *aabb,
                                                    double *B2v, const uint32_t *lstart, int level,
                                                    int64_t nnmax) {
    const uint32_t b0 = lstart[level], b1 = lstart[level + 1];
    for (uint32_t b = b0 + blockIdx.x * 256 + threadIdx.x; b < b1; b += gridDim.x * 256) {
        Node &N = node[b];
        const uint32_t nch = N.meta & 255u;
        double M = 0.0, s[3] = {0.0, 0.0, 0.0};
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (nch == 0) {
            for (uint32_t i = N.first; i < N.first + N.count; i++) {
                for (int a = 0; a < 3; a++) {
                    const double v = x[a * n + i];
                    lo[a] = fmin(lo[a], v);
                    hi[a] = fmax(hi[a], v);
                }
                if (MOM) {
                    const double4 q = src[i];
                    M += q.w;
                    s[0] = fma(q.w, q.x, s[0]);
                    s[1] = fma(q.w, q.y, s[1]);
                    s[2] = fma(q.w, q.z, s[2]);
                }
            }
        } else {
            for (uint32_t k = 0; k < nch; k++) {
                const uint32_t c = N.child + k;
                for (int a = 0; a < 3; a++) {
                    lo[a] = fmin(lo[a], aabb[8 * (int64_t)c + a]);
                    hi[a] = fmax(hi[a], aabb[8 * (int64_t)c + 4 + a]);
                }
                if (MOM) {
                    M += node[c].M;
                    for (int a = 0; a < 3; a++) s[a] += S3[a * nnmax + c];
                }
            }
        }
        store_box(aabb, b, lo, hi);
        if (MOM) {
            N.M = M;
            for (int a = 0; a < 3; a++) {
                S3[a * nnmax + b] = s[a];
                N.com[a] = (M != 0.0) ? s[a] / M : N.blo[a] + 0.5 * N.l;
            }
        }
        if (MAC) {
            const double com[3] = {N.com[0], N.com[1], N.com[2]};
            double B2 = 0.0;
            if (nch == 0) {
                for (uint32_t i = N.first; i < N.first + N.count; i++) {
                    const double4 q = src[i];
                    B2 = fma(q.w, sqdist(com, q.x, q.y, q.z), B2);
                }
            } else {
                for (uint32_t k = 0; k < nch; k++) {
                    const Node &C = node[N.child + k];
                    B2 = B2 + fma(C.M, sqdist(com, C.com[0], C.com[1], C.com[2]), B2v[N.child + k]);
                }
            }
            B2v[b] = B2;
        }
    }
}

// b_max^2 = max |COM - u|^2 over a node's particles (a maximum, exact in
// any order).  Nodes of at most kBmaxSmall particles are done by one thread
// each; the others are cut into chunks of kBmaxChunk particles, one wave per
// chunk, combined with atomic maxima on the bits of the (non-negative)
// doubles.
constexpr uint32_t kBmaxSmall = 256, kBmaxChunk = 4096;

__global__ __launch_bounds__(256) void k_bmax_small(const Node *node, const uint32_t *nn_dev,
                                                    const double4 *src, int64_t nnmax,
                                                    unsigned long long *bmax, uint32_t *items) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    const uint32_t nn = *nn_dev;
    if (b > (uint32_t)nnmax) return;
    if (b >= nn) {
        items[b] = 0u;       // the scan runs over nnmax + 1 entries
        return;
    }
    const Node &N = node[b];
    if (N.count > kBmaxSmall) {
        items[b] = (N.count + kBmaxChunk - 1) / kBmaxChunk;
        bmax[b] = 0ull;
        return;
    }
    items[b] = 0u;
    const double com[3] = {N.com[0], N.com[1], N.com[2]};
    // eight particles loaded ahead of their use (a maximum is exact in any
    // order): a node of 256 particles waits for 32 rounds of loads, not 256
    const uint32_t f = N.first, e = N.first + N.count;
    double m = 0.0;
    for (uint32_t i0 = f; i0 < e; i0 += 8) {
        double4 q[8];
#pragma unroll
        for (int j = 0; j < 8; j++) q[j] = src[i0 + j < e ? i0 + j : i0];
#pragma unroll
        for (int j = 0; j < 8; j++) m = fmax(m, sqdist(com, q[j].x, q[j].y, q[j].z));
    }
    bmax[b] = (unsigned long long)__double_as_longlong(m);
}

// items holds the exclusive scan of the chunk counts; total their sum.
__global__ __launch_bounds__(256) void k_bmax_big(const Node *node, const uint32_t *nn_dev,
                                                  const double4 *src, const uint32_t *items,
                                                  const uint32_t *total,
                                                  unsigned long long *bmax) {
    const uint32_t nn = *nn_dev, nw = *total;
    const int lane = __lane_id();
    for (uint32_t w = blockIdx.x * 4 + (threadIdx.x >> 6); w < nw; w += gridDim.x * 4) {
        // the node owning work item w: the last with items[b] <= w (nodes
        // without chunks share their offset with the next node, which has
        // the chunks)
        uint32_t lo = 0, hi = nn;      // items[lo] <= w < items[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (items[mid] <= w) lo = mid; else hi = mid;
        }
        const Node &N = node[lo];
        const uint32_t k = w - items[lo];
        const uint32_t i0 = N.first + k * kBmaxChunk;
        const uint32_t e = N.first + N.count;
        const uint32_t i1 = e < i0 + kBmaxChunk ? e : i0 + kBmaxChunk;
        const double com[3] = {N.com[0], N.com[1], N.com[2]};
        double m = 0.0;
        for (uint32_t i = i0 + (uint32_t)lane; i < i1; i += 64) {
            const double4 q = src[i];
            m = fmax(m, sqdist(com, q.x, q.y, q.z));
        }
        m = wave_max(m);
        if (lane == 0) atomicMax(&bmax[lo], (unsigned long long)__double_as_longlong(m));
    }
}

// Absolute MAC (section II.B eq. 5) for the nodes of systems with a_err > 0:
// b = sqrt(bmax2), t = sqrt(((3 G) B2) / a_err), r_b = 0.5 b + sqrt(0.25
// bmax2 + t), rb2 = r_b * r_b; every sqrt and the division correctly
// rounded.  Other systems keep l^2 / theta^2.
__global__ __launch_bounds__(256) void k_abs_mac(Node *node, const uint32_t *nn_dev,
                                                 const Sys *sys, const double *B2v,
                                                 const unsigned long long *bmax) {
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= *nn_dev) return;
    Node &N = node[b];
    const Sys &y = sys[N.sys];
    if (!(y.aerr > 0.0)) return;
    const double bm = __longlong_as_double((long long)bmax[b]);
    const double t = sqrt(((3.0 * y.G) * B2v[b]) / y.aerr);
    const double rb = 0.5 * sqrt(bm) + sqrt(0.25 * bm + t);
    N.rb2 = rb * rb;
}

// Refit after a drift (same tree, same sorted order): node boxes directly
// from their particle ranges, which needs no level order.  Boxes of aligned
// chunks of 32, 32^2 and 32^3 sorted particles are reduced first; a node's
// range is then covered by the largest aligned chunks that fit (at most 31
// pieces of each size on either side), kRefitLanes lanes per node, nodes in
// pre-order.  Minima and maxima are exact, so the boxes equal those of the
// level pass.
constexpr int kC1 = 32;

// dst[6][ceil(m / 32)]: boxes of 32 consecutive entries of src (particles
// when src6 is null: x [3][m], else boxes src6 [6][m]).
__global__ __launch_bounds__(256) void k_box32(const double *x, const double *src6, int64_t m,
                                               double *dst, int64_t md) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = i < m;
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        if (src6) {
            lo[a] = in ? src6[a * m + i] : INFINITY;
            hi[a] = in ? src6[(3 + a) * m + i] : -INFINITY;
        } else {
            const double v = in ? x[a * m + i] : 0.0;
            lo[a] = in ? v : INFINITY;
            hi[a] = in ? v : -INFINITY;
        }
        for (int o = 16; o > 0; o >>= 1) {     // within each half wavefront
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
        }
    }
    const int64_t c = i / kC1;
    if ((threadIdx.x & (kC1 - 1)) == 0 && c < md)
        for (int a = 0; a < 3; a++) {
            dst[a * md + c] = lo[a];
            dst[(3 + a) * md + c] = hi[a];
        }
}

constexpr int kRefitLanes = 4;   // lanes per node in k_refit

__global__ __launch_bounds__(256) void k_refit(const Node *node, const uint32_t *nn_dev,
                                               const uint32_t *pre2bfs, const double *x,
                                               int64_t n, const double *c1, int64_t m1,
                                               const double *c2, int64_t m2, const double *c3,
                                               int64_t m3, double *aabb, int64_t nnmax) {
    // kRefitLanes consecutive lanes per node, nodes in pre-order, so
    // neighbouring lanes hold leaves with adjacent particle ranges and their
    // loads share cache lines; the node's lanes return together, so the
    // shuffles below read only lanes that are still running
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    const uint32_t p = t / kRefitLanes, sub = t % kRefitLanes;
    if (p >= *nn_dev) return;
    const uint32_t b = pre2bfs[p];
    const uint32_t f = node[b].first, e = f + node[b].count;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    // [f, e) = singles | 32-chunks | 1024-chunks | 32768-chunks | 1024 | 32 | singles,
    // each run aligned to its chunk size (min and max are exact, so any cover
    // gives the same box); every run is a counted loop in which the node's
    // lanes take every kRefitLanes-th piece, each lane four pieces at a time
    constexpr uint32_t L = kRefitLanes;
    auto run = [&](const double *c, int64_t m, uint32_t k0, uint32_t k1) {
        for (uint32_t k = k0 + sub; k < k1; k += 4 * L) {
            double l4[4][3], h4[4][3];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t kk = k + j * L < k1 ? k + j * L : k;
                for (int a = 0; a < 3; a++) {
                    l4[j][a] = c[a * m + kk];
                    h4[j][a] = c[(3 + a) * m + kk];
                }
            }
#pragma unroll
            for (int j = 0; j < 4; j++)
                for (int a = 0; a < 3; a++) {
                    lo[a] = fmin(lo[a], l4[j][a]);
                    hi[a] = fmax(hi[a], h4[j][a]);
                }
        }
    };
    auto singles = [&](uint32_t i0, uint32_t i1) {
        for (uint32_t i = i0 + sub; i < i1; i += 4 * L) {
            double v4[4][3];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t ii = i + j * L < i1 ? i + j * L : i;
                for (int a = 0; a < 3; a++) v4[j][a] = x[a * n + ii];
            }
#pragma unroll
            for (int j = 0; j < 4; j++)
                for (int a = 0; a < 3; a++) {
                    lo[a] = fmin(lo[a], v4[j][a]);
                    hi[a] = fmax(hi[a], v4[j][a]);
                }
        }
    };
    constexpr uint32_t S1 = kC1, S2 = kC1 * kC1, S3 = kC1 * kC1 * kC1;
    const uint32_t a1 = (f + S1 - 1) / S1 * S1, b1 = e / S1 * S1;
    if (a1 >= b1) {
        singles(f, e);
    } else {
        singles(f, a1);
        singles(b1, e);
        const uint32_t a2 = (a1 + S2 - 1) / S2 * S2, b2 = b1 / S2 * S2;
        if (a2 >= b2) {
            run(c1, m1, a1 / S1, b1 / S1);
        } else {
            run(c1, m1, a1 / S1, a2 / S1);
            run(c1, m1, b2 / S1, b1 / S1);
            const uint32_t a3 = (a2 + S3 - 1) / S3 * S3, b3 = b2 / S3 * S3;
            if (a3 >= b3) {
                run(c2, m2, a2 / S2, b2 / S2);
            } else {
                run(c2, m2, a2 / S2, a3 / S2);
                run(c2, m2, b3 / S2, b2 / S2);
                run(c3, m3, a3 / S3, b3 / S3);
            }
        }
    }
    for (int o = 1; o < (int)L; o <<= 1)
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
        }
    if (sub == 0) store_box(aabb, b, lo, hi);
}

// Sizes of the three chunk levels for n particles (entries of 6 doubles).
void refit_sizes(int64_t n, int64_t *m1, int64_t *m2, int64_t *m3) {
    *m1 = (n + kC1 - 1) / kC1;
    *m2 = (*m1 + kC1 - 1) / kC1;
    *m3 = (*m2 + kC1 - 1) / kC1;
}

void launch_refit(BuildBufs &B, hipStream_t s) {
    const int64_t n = B.n;
    int64_t m1, m2, m3;
    refit_sizes(n, &m1, &m2, &m3);
    double *c1 = B.cbox, *c2 = c1 + 6 * m1, *c3 = c2 + 6 * m2;
    const double *x = B.x[B.cur];
    hipLaunchKernelGGL(k_box32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, nullptr, n,
                       c1, m1);
    hipLaunchKernelGGL(k_box32, dim3((unsigned)((m1 + 255) / 256)), dim3(256), 0, s, nullptr, c1,
                       m1, c2, m2);
    hipLaunchKernelGGL(k_box32, dim3((unsigned)((m2 + 255) / 256)), dim3(256), 0, s, nullptr, c2,
                       m2, c3, m3);
    hipLaunchKernelGGL(k_refit, dim3((unsigned)((kRefitLanes * B.nnmax + 255) / 256)), dim3(256),
                       0, s, B.node, B.nn, B.pre2bfs, x, n, c1, m1, c2, m2, c3, m3, B.aabb,
                       B.nnmax);
}

// The bottom-up pass over all levels (lstart must be current): node boxes,
// and moments if asked.  Also the refit of the boxes after a drift.
void launch_levels(BuildBufs &B, bool moments, hipStream_t s) {
    unsigned gn = (unsigned)((B.nnmax + 255) / 256);
    unsigned gl = gn < 1024u ? gn : 1024u;
    const double *x = B.x[B.cur];
    const bool mac = moments && B.abs_mac;
    for (int l = kMaxLevel; l >= 0; l--) {
        if (mac)
            hipLaunchKernelGGL((k_level_pass<true, true>), dim3(gl), dim3(256), 0, s, B.node,
                               B.src, x, B.n, B.S3, B.aabb, B.B2, B.lstart, l, B.nnmax);
        else if (moments)
            hipLaunchKernelGGL((k_level_pass<true, false>), dim3(gl), dim3(256), 0, s, B.node,
                               B.src, x, B.n, B.S3, B.aabb, B.B2, B.lstart, l, B.nnmax);
        else
            hipLaunchKernelGGL((k_level_pass<false, false>), dim3(gl), dim3(256), 0, s, B.node,
                               B.src, x, B.n, B.S3, B.aabb, B.B2, B.lstart, l, B.nnmax);
    }
    if (mac) {
        // b_max^2, then the opening radii of the absolute MAC
        const unsigned gi = (unsigned)((B.nnmax + 1 + 255) / 256);
        hipLaunchKernelGGL(k_bmax_small, dim3(gi), dim3(256), 0, s, B.node, B.nn, B.src, B.nnmax,
                           B.bmax, B.bitems);
        launch_scan_u32(B.bitems, B.nnmax + 1, B.scan_part, B.nn + 2, s);
        // chunks: at most n / kBmaxChunk per level plus one per big node
        const int64_t most = (B.n / kBmaxChunk + 1) * (kMaxLevel + 1) + B.n / kBmaxSmall + 1;
        const int64_t nb = (most + 3) / 4;
        hipLaunchKernelGGL(k_bmax_big, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(256), 0, s,
                           B.node, B.nn, B.src, B.bitems, B.nn + 2, B.bmax);
        hipLaunchKernelGGL(k_abs_mac, dim3(gn), dim3(256), 0, s, B.node, B.nn, B.sys, B.B2,
                           B.bmax);
    }
}

void launch_topology(BuildBufs &B, bool moments, hipStream_t s) {
    int64_t n = B.n;
    unsigned gb = (unsigned)((n + 255) / 256);
    const uint64_t *key = B.key[0];
    int8_t *dwin = (int8_t *)B.lvl_key2;   // scratch: reused for the partitioned keys later
    hipLaunchKernelGGL(k_cpl, dim3(gb), dim3(256), 0, s, key, n, B.sys_of, B.sys, B.cpl, dwin);
    hipLaunchKernelGGL(k_leaflev, dim3(gb), dim3(256), 0, s, B.cpl, dwin, n, B.sys_of, B.sys,
                       B.leaflev, B.nstart);
    launch_scan_u32(B.nstart, n + 1, B.scan_part, B.nn, s);
    hipLaunchKernelGGL(k_emit_pre, dim3(gb), dim3(256), 0, s, B.cpl, B.nstart, n, B.sys_of,
                       B.sysbits, B.pre_key, B.pre_val, B.pre_first);
    {
        const int64_t nb = (B.nnmax + 255) / 256;
        hipLaunchKernelGGL(k_node_count, dim3((unsigned)(nb < 2048 ? nb : 2048)), dim3(256), 0, s,
                           key, B.pre_key, B.pre_first, B.nn, B.sys, B.sysbits, B.pre_count);
    }
    // stable partition by (level, system): 5 + sysbits key bits
    const int kbits = 5 + B.sysbits;
    int64_t nb = sort_blocks(B.nnmax);
    if (nb < 1) nb = 1;
    uint32_t *hpart = B.hist + 256 * nb;
    uint32_t *kin = B.pre_key, *vin = B.pre_val;
    const int npass = (kbits + 7) / 8;
    for (int pass = 0; pass < npass; pass++) {
        const bool last = pass == npass - 1;
        uint32_t *kout = last ? B.lvl_key2 : (kin == B.ptmp_k ? B.pre_key : B.ptmp_k);
        uint32_t *vout = last ? B.bfs2pre : (vin == B.ptmp_v ? B.pre_val : B.ptmp_v);
        radix_pass<uint32_t>(kin, vin, kout, vout, B.hist, hpart, B.nn, B.nnmax, 8 * pass, s);
        kin = kout;
        vin = vout;
    }
    unsigned gn = (unsigned)((B.nnmax + 255) / 256);
    hipLaunchKernelGGL(k_pre2bfs, dim3(gn), dim3(256), 0, s, B.bfs2pre, B.nn, B.pre2bfs);
    hipLaunchKernelGGL(k_fill_nodes, dim3(gn), dim3(256), 0, s, key, B.leaflev, B.nstart,
                       B.bfs2pre, B.pre2bfs, B.lvl_key2, B.pre_first, B.pre_count, B.nn, B.frame,
                       B.sys, B.sysbits, B.node);
    hipLaunchKernelGGL(k_level_starts, dim3(gn), dim3(256), 0, s, B.lvl_key2, B.sysbits, B.nn,
                       B.lstart);
    launch_levels(B, moments, s);
}

// ---------------------------------------------------------------------------
// sink groups.  Soft groups (the same rule as the tree contract; g is the
// system's group size, L = gcell * g its chunking limit): the chunking cells
// -- cells of at most L particles whose parent holds more (the root if it is
// that small), and leaves whose parent holds more -- are cut into
// consecutive chunks of g.  Hard groups
// (the hard kernel's own table; any partition gives the same neighbour sets):
// a cell with at most g particles is a group; a bigger cell is split into its
// children; where all children are small, consecutive children are packed
// while the total stays <= g; a bigger leaf is cut into chunks of g.  Each
// node marks the group starts it owns; a scan turns the marks into a table.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_soft_group_marks(const Node *node, const uint32_t *nn_dev,
                                                          const Sys *sys, uint32_t *flag) {
    uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= *nn_dev) return;
    const Node &N = node[b];
    const uint32_t g = sys[N.sys].g, lim = sys[N.sys].gcell * g;
    const uint32_t count = N.count, nch = N.meta & 255u;
    if (count > lim && nch != 0) return;                        // split further
    if ((N.meta >> 8) != 0 && node[N.parent].count <= lim) return;   // inside a chunking cell
    for (uint32_t s = 0; s < count; s += g) flag[N.first + s] = 1u;
}

__global__ __launch_bounds__(256) void k_group_marks(const Node *node, const uint32_t *nn_dev,
                                                     const Sys *sys, uint32_t *flag) {
    uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= *nn_dev) return;
    const Node &N = node[b];
    const uint32_t g = sys[N.sys].g;
    uint32_t count = N.count, nch = N.meta & 255u;
    if (count <= g) {
        if ((N.meta >> 8) == 0) flag[N.first] = 1u;   // a small root is one group
        return;
    }
    if (nch == 0) {
        for (uint32_t s = 0; s < count; s += g) flag[N.first + s] = 1u;
        return;
    }
    bool pack = true;
    for (uint32_t k = 0; k < nch; k++) pack &= node[N.child + k].count <= g;
    uint32_t run = 0;
    for (uint32_t k = 0; k < nch; k++) {
        const Node &C = node[N.child + k];
        if (C.count > g) continue;      // split by its own thread
        if (!pack) {
            flag[C.first] = 1u;
            continue;
        }
        if (run > 0 && run + C.count > g) run = 0;
        if (run == 0) flag[C.first] = 1u;
        run += C.count;
    }
}

__global__ __launch_bounds__(256) void k_group_compact(const uint32_t *scan, int64_t n,
                                                       uint32_t *gstart) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t s = scan[i];
    if (scan[i + 1] != s) gstart[s] = (uint32_t)i;
    if (i == n - 1) gstart[scan[n]] = (uint32_t)n;
}

void launch_groups(BuildBufs &B, hipStream_t s) {
    int64_t n = B.n;
    unsigned gn = (unsigned)((B.nnmax + 255) / 256);
    unsigned gp = (unsigned)((n + 255) / 256);
    // soft groups; the flags live in nstart, free once the topology is built
    uint32_t *flag = B.nstart;
    launch_zero_u32(flag, n + 1, s);
    hipLaunchKernelGGL(k_soft_group_marks, dim3(gn), dim3(256), 0, s, B.node, B.nn, B.sys, flag);
    launch_scan_u32(flag, n + 1, B.scan_part, B.ng, s);
    hipLaunchKernelGGL(k_group_compact, dim3(gp), dim3(256), 0, s, flag, n, B.gstart);
    // hard groups; flags in pre_key (nnmax >= n + 1 entries, free after the build)
    uint32_t *hflag = B.pre_key;
    launch_zero_u32(hflag, n + 1, s);
    hipLaunchKernelGGL(k_group_marks, dim3(gn), dim3(256), 0, s, B.node, B.nn, B.sys, hflag);
    launch_scan_u32(hflag, n + 1, B.scan_part, B.nhg, s);
    hipLaunchKernelGGL(k_group_compact, dim3(gp), dim3(256), 0, s, hflag, n, B.hgstart);
}

}  // namespace htree
