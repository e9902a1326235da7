// force.hip -- soft (tree) and hard (neighbour) force kernels for gfx950.
//
// Soft force (section II.B walk, grouped sinks of section III.A.2, split of
// section II.C).  One wavefront serves one sink group (at most 64 sinks,
// consecutive in key order inside one cell), one sink per lane.  The walk is
// wide depth-first over a stack of child ranges (first node, count) in LDS:
// each step takes up to 64 nodes from the top ranges, one per lane, and tests
// them in FP64 against the group's bounding box:
//   D1 = dist^2(box_g, COM),  D2 = dist^2(box_g, cell box)
//   accepted iff D1 >= r_b^2 and (hybrid ? D2 >= R2^2 : D2 > 0),
// with r_b = l / theta or the absolute MAC of section II.B (computed by the
// build); with the paper's group rule (MINS) a cell the box test would open is
// measured again by its nearest sink, min_i |u_i - COM|^2, instead of D1.
// Accepted cells become particle-cell sources, rejected leaves particle
// sources ("near", weighted by 1 - K, iff hybrid and D2 < R2^2), other nodes
// push the range of their (contiguous) children.  Sources are staged in LDS as
// offsets from the group centre plus mass; every 64 of them all lanes run the
// interaction loop, per tile in FP32 (precision 0) or FP64 (precision 1),
// tiles merged with compensated (Kahan) summation; a near source's weight is
// evaluated only when some lane has it within R2 (beyond, it is exactly 1).
// No list leaves the chip.
//
// The stack stays bounded: every popped node pushes at most one range, so a
// step may take `want` nodes only while top + want leaves a reserve of 22
// entries; past that the walk takes one node at a time, depth first, which
// keeps at most one partial range per tree level (21).
//
// Groups are dealt to workgroups by the hardware dispatcher (see sched_group):
// one workgroup per group for the expected group count, a grid-stride loop
// beyond it.  Work item positions map to groups through a dispatch order
// (heaviest estimated cost first, built by the library between launches), so
// that expensive groups do not start last and leave a tail.
//
// Hard force (section II.C, eq. 10): per group, a walk that opens every node
// whose box (the bounding box of its particles' master positions, kept
// current by a refit after each drift) lies within R2 (plus rounding slack)
// of the group box collects candidate leaves into a batch; the batch's
// particles are gathered in a stride order that mixes the leaves (LeafOrder)
// and filtered against the group box, then every candidate pair is decided
// by the exact FP64 test fma(dz,dz, fma(dy,dy, dx*dx)) < R2^2 on the master
// positions, and accepted pairs add K(r) times the softened pair force, in
// FP64.  The hard kernel has its own group table (cells of at most 64
// particles) and gathers one packed record (x, y, z, m) per particle.  With
// search reuse, the first launch after a build records each group's walk and
// the launches after refits replay it (hard_group<MODE>).
#include "htree_dev.h"

#include <math.h>

namespace htree {

constexpr int kStk = 448;          // range entries (16 workgroups of LDS fit a CU)
constexpr int kStkReserve = 22;    // depth-first progress room (one range per level)
constexpr int kPC = 128;
constexpr int kRQ = 128;

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Arithmetic of the soft interactions: FP32 (precision 0) or FP64
// (precision 1).  Sources are staged as offsets from the group centre in that
// type, with the mass.
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;

__device__ inline float4 make_vec4(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
__device__ inline double4 make_vec4(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
}

// 1/sqrt: the hardware FP32 estimate, or in FP64 from that seed with two
// Newton steps (relative error near the FP64 rounding).
__device__ inline float rsqrt_t(float x) { return rsq(x); }
__device__ inline double rsqrt_t(double x) {
    double y = (double)rsq((float)x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    return y * fma(-0.5 * x, y * y, 1.5);
}
__device__ inline float sqrt_t(float x) { return fsqrt(x); }
__device__ inline double sqrt_t(double x) { return x > 0.0 ? x * rsqrt_t(x) : 0.0; }
__device__ inline float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float clamp01(float y) { return fminf(fmaxf(y, 0.0f), 1.0f); }
__device__ inline double clamp01(double y) { return fmin(fmax(y, 0.0), 1.0); }


__device__ inline double gap_pt(double lo, double hi, double p) {
    double g = fmax(lo - p, p - hi);
    return g > 0.0 ? g : 0.0;
}
__device__ inline double gap_box(double glo, double ghi, double clo, double chi) {
    double g = fmax(glo - chi, clo - ghi);
    return g > 0.0 ? g : 0.0;
}
__device__ inline double dist2(double gx, double gy, double gz) {
    return fma(gz, gz, fma(gy, gy, gx * gx));
}

// 1 - K(r) as a polynomial in w = 1 - Y^2 (K(Y) = S(Y^2) with the quintic
// S(s) = 10 s^3 - 15 s^4 + 6 s^5, and 1 - S(s) = S(1 - s)).
template <typename T>
__device__ inline T one_minus_K(T r, T R2, T invdR) {
    const T Y = clamp01((R2 - r) * invdR);
    T w = fma_t(-Y, Y, (T)1);
    T t = fma_t(fma_t((T)6, w, (T)-15), w, (T)10);
    return t * (w * w * w);
}

__device__ inline double K_of64(double r, double R2, double invdR) {
    double Y = (R2 - r) * invdR;
    Y = fmin(fmax(Y, 0.0), 1.0);
    double s = Y * Y;
    double t = fma(fma(6.0, s, -15.0), s, 10.0);
    return t * (s * s * s);
}

// Work distribution.  Each workgroup (one wavefront) serves the groups
// idx = blockIdx.x + k * gridDim.x, with gridDim.x a multiple of 8.  The
// dispatcher deals workgroups to the 8 XCDs round-robin (XCD = blockIdx % 8)
// and, within an XCD, starts them in index order as slots free up, so a slow
// group does not hold back the others.  sched_group maps work item idx to a
// group so that each XCD takes runs of kRun consecutive groups (which share
// tree nodes and particles in that XCD's L2), interleaved with the other XCDs
// at a period of 8 * kRun groups (so the dense regions of a system, which are
// contiguous in key order, are spread over all XCDs).  The map is a bijection
// of [0, ng): a permutation inside each full period, the identity on the tail.
constexpr uint32_t kRun = 16;

__device__ inline uint32_t sched_group(uint32_t idx, uint32_t ng) {
    constexpr uint32_t period = 8 * kRun;
    const uint32_t full = ng - ng % period;
    if (idx >= full) return idx;
    const uint32_t r = idx % period;
    return idx - r + (r % 8) * kRun + r / 8;
}

// Capacity guard of the walks' LDS queues (wave-uniform `over`).  The
// bounds are kept by construction, so this never fires; if it did, the
// context's status word would report HTREE_EOVERFLOW (htree_sync) and the
// caller drops the group's remaining work instead of writing past a queue.
__device__ inline bool over_capacity(uint32_t *status, bool over) {
    if (over && __lane_id() == 0) atomicOr(status, kStatusOverflow);
    return over;
}

// A wave-uniform double held in scalar registers.
__device__ inline double uniform_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// First counter of this workgroup's tally slot.
__device__ inline int tally_slot() { return (int)(blockIdx.x % kTallySlots) * kTallyStride; }

__global__ void k_tally_fold(const unsigned long long *slots, unsigned long long *sum) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    unsigned long long t = 0;
    for (int j = 0; j < kTallySlots; j++) t += slots[j * kTallyStride + k];
    sum[k] = t;
}

void launch_tally_fold(const unsigned long long *slots, unsigned long long *sum, hipStream_t s) {
    hipLaunchKernelGGL(k_tally_fold, dim3(1), dim3(64), 0, s, slots, sum);
}

// Group setup shared by both walks.
struct GroupCtx {
    uint32_t b0;
    uint32_t sys;       // system of the group; its root is node `sys`
    int ns;
    bool act;
    double lo[3], hi[3], c[3];
};

__device__ inline void group_setup(const double4 *src, const uint32_t *gstart,
                                   const uint32_t *sys_of, uint32_t grp, GroupCtx &G,
                                   double4 &me) {
    const int lane = __lane_id();
    G.b0 = gstart[grp];
    G.sys = sys_of[G.b0];
    G.ns = (int)(gstart[grp + 1] - G.b0);
    G.act = lane < G.ns;
    me = src[G.act ? G.b0 + lane : G.b0];
    double p[3] = {me.x, me.y, me.z};
    for (int a = 0; a < 3; a++) {
        G.lo[a] = uniform_f64(wave_min(p[a]));
        G.hi[a] = uniform_f64(wave_max(p[a]));
        G.c[a] = 0.5 * (G.lo[a] + G.hi[a]);
    }
}

// A source particle as an offset from the group centre, with its mass.
template <typename T>
__device__ inline vec4_t<T> rel_src(const double4 &q, const GroupCtx &G) {
    return make_vec4((T)(q.x - G.c[0]), (T)(q.y - G.c[1]), (T)(q.z - G.c[2]), (T)q.w);
}

// ---------------------------------------------------------------------------
// interaction loops
// ---------------------------------------------------------------------------
template <typename T>
struct Acc {
    T a[3], c[3];   // running sums and Kahan compensations
    T p, pc;
};

template <typename T>
__device__ inline void kahan(T &s, T &c, T v) {
    T y = v - c;
    T t = s + y;
    c = (t - s) - y;
    s = t;
}

template <bool POT, typename T>
__device__ inline void far_pair(const vec4_t<T> &q, T sx, T sy, T sz, T eps2, T &ax, T &ay, T &az,
                                T &ph) {
    T dx = q.x - sx, dy = q.y - sy, dz = q.z - sz;
    T r2 = fma_t(dz, dz, fma_t(dy, dy, fma_t(dx, dx, eps2)));
    T ri = rsqrt_t(r2);
    T mr = q.w * ri;
    T f = mr * (ri * ri);
    ax = fma_t(f, dx, ax);
    ay = fma_t(f, dy, ay);
    az = fma_t(f, dz, az);
    if (POT) ph -= mr;
}

template <bool POT, int CNT, typename T>
__device__ inline void eval_far(const vec4_t<T> *t, int cnt, T sx, T sy, T sz, T eps2, Acc<T> &A) {
    // two accumulator sets (even and odd sources) halve the dependent chain
    T ax = 0, ay = 0, az = 0, ph = 0, bx = 0, by = 0, bz = 0, pb = 0;
    const int nloop = CNT > 0 ? CNT : cnt;
    int j = 0;
#pragma unroll 4
    for (; j + 2 <= nloop; j += 2) {
        const vec4_t<T> q = t[j], p = t[j + 1];
        far_pair<POT, T>(q, sx, sy, sz, eps2, ax, ay, az, ph);
        far_pair<POT, T>(p, sx, sy, sz, eps2, bx, by, bz, pb);
    }
    if (j < nloop) far_pair<POT, T>(t[j], sx, sy, sz, eps2, ax, ay, az, ph);
    ax += bx;
    ay += by;
    az += bz;
    ph += pb;
    kahan(A.a[0], A.c[0], ax);
    kahan(A.a[1], A.c[1], ay);
    kahan(A.a[2], A.c[2], az);
    if (POT) kahan(A.p, A.pc, ph);
}

// Near sources (leaves within R2 of the group box): the weight 1 - K(r).
// Most of their pairs lie beyond R2, where 1 - K is exactly 1 (Y clamps to
// 0, so w = 1 and the polynomial gives 1); u2skip is R2^2 raised by a margin
// above the rounding of the square root, so a source for which every lane
// has u^2 >= u2skip is summed without the weight (and without its square
// root) and every result is the same as with it.
template <bool POT, typename T>
__device__ inline void near_pair(const vec4_t<T> &q, T sx, T sy, T sz, T eps2, T R2, T invdR,
                                 T u2skip, T &ax, T &ay, T &az, T &ph) {
    T dx = q.x - sx, dy = q.y - sy, dz = q.z - sz;
    T u2 = fma_t(dz, dz, fma_t(dy, dy, dx * dx));
    T ri = rsqrt_t(u2 + eps2);
    T mr = q.w * ri;
    T f = mr * (ri * ri);
    if (__ballot(u2 < u2skip)) f = f * one_minus_K(sqrt_t(u2), R2, invdR);
    ax = fma_t(f, dx, ax);
    ay = fma_t(f, dy, ay);
    az = fma_t(f, dz, az);
    if (POT) ph -= mr;
}

template <bool POT, typename T>
__device__ inline void eval_near(const vec4_t<T> *t, int cnt, T sx, T sy, T sz, T eps2, T R2,
                                 T invdR, T u2skip, Acc<T> &A) {
    T ax = 0, ay = 0, az = 0, ph = 0;
    int j = 0;
    // eight sources loaded ahead of their (branching) evaluation
    for (; j + 8 <= cnt; j += 8) {
        vec4_t<T> q[8];
#pragma unroll
        for (int r = 0; r < 8; r++) q[r] = t[j + r];
#pragma unroll
        for (int r = 0; r < 8; r++)
            near_pair<POT, T>(q[r], sx, sy, sz, eps2, R2, invdR, u2skip, ax, ay, az, ph);
    }
    for (; j < cnt; j++)
        near_pair<POT, T>(t[j], sx, sy, sz, eps2, R2, invdR, u2skip, ax, ay, az, ph);
    kahan(A.a[0], A.c[0], ax);
    kahan(A.a[1], A.c[1], ay);
    kahan(A.a[2], A.c[2], az);
    if (POT) kahan(A.p, A.pc, ph);
}

// Takes `want` items from the top of a range stack (nr ranges, each count
// >= 1, the top 64 ranges holding at least `want` items), consuming each range
// from its end.  Range q (0 = bottom) is held in first[O.slot(q)],
// cnt[O.slot(q)].  Returns this lane's item (lane < want).  All lanes must
// call it.
template <typename Order>
__device__ inline uint32_t take_items(uint32_t *first, uint32_t *cnt, int &nr, int want,
                                      uint32_t *scan, const Order &O) {
    const int lane = __lane_id();
    HT_CHECK(want >= 1 && want <= 64 && nr >= 1);
    int r = nr < 64 ? nr : 64;
    uint32_t ck = lane < r ? cnt[O.slot(nr - 1 - lane)] : 0u;
    uint32_t inc = wave_incl_scan(ck);
    const uint32_t exc = inc - ck;
    // item j belongs to the last range starting at or before j: each range
    // marks its start (start << 8 | index + 1), a running maximum over the
    // lanes carries the mark to the items after it
    scan[lane] = 0u;
    __syncthreads();
    if (lane < r && exc < 64u) scan[exc] = (exc << 8) | (uint32_t)(lane + 1);
    __syncthreads();
    const uint32_t own = wave_incl_max(scan[lane]);
    uint32_t item = 0;
    if (lane < want) {
        const int k = (int)(own & 255u) - 1;
        const uint32_t prev = own >> 8;
        const int sl = O.slot(nr - 1 - k);
        uint32_t f = first[sl], c = cnt[sl];
        item = f + c - 1u - ((uint32_t)lane - prev);
    }
    HT_CHECK(__shfl(inc, r - 1) >= (uint32_t)want);
    uint64_t full = __ballot(lane < r && inc <= (uint32_t)want);
    int nfull = __popcll(full);
    uint32_t used = nfull ? (uint32_t)__builtin_amdgcn_readlane(inc, nfull - 1) : 0u;
    __syncthreads();
    if (lane == 0 && (uint32_t)want > used) cnt[O.slot(nr - 1 - nfull)] -= (uint32_t)want - used;
    nr -= nfull;
    __syncthreads();
    return item;
}

// Ranges stored in stack order: position q is entry q.
struct StackOrder {
    __device__ int slot(int q) const { return q; }
};

__device__ inline uint32_t take_items(uint32_t *first, uint32_t *cnt, int &nr, int want,
                                      uint32_t *scan) {
    return take_items(first, cnt, nr, want, scan, StackOrder{});
}

// Number of nodes a walk step may take: up to 64, keeping room for one pushed
// range per popped node plus the depth-first reserve.
__device__ inline int step_width(int top, uint32_t avail) {
    int w = avail < 64u ? (int)avail : 64;
    int room = kStk - kStkReserve - top;
    if (w > room) w = room > 1 ? room : 1;
    return w;
}

// ---------------------------------------------------------------------------
// soft force
// ---------------------------------------------------------------------------
template <typename T>
struct SoftLDS {
    uint32_t sfirst[kStk], scnt[kStk];
    vec4_t<T> pc[kPC];
    vec4_t<T> tile[2][64];
    uint32_t ffirst[kRQ], fcnt[kRQ];
    uint32_t nfirst[kRQ], ncnt[kRQ];
    uint32_t scan[64];
};

// Per-system constants of the interactions in the arithmetic type.
struct SoftConst32 {
    float eps2, R2, invdR, G;
    __device__ SoftConst32(const SysF &P) : eps2(P.eps2), R2(P.R2f), invdR(P.invdR), G(P.G) {}
};
struct SoftConst64 {
    double eps2, R2, invdR, G;
    __device__ SoftConst64(const SysF &P) : eps2(P.eps2d), R2(P.R2d), invdR(P.invdR64), G(P.Gd) {}
};
template <typename T> struct SoftConst;
template <> struct SoftConst<float> : SoftConst32 { using SoftConst32::SoftConst32; };
template <> struct SoftConst<double> : SoftConst64 { using SoftConst64::SoftConst64; };

template <bool HYBRID, bool POT, bool MINS, typename T>
__device__ void soft_group(const ForceArgs &A, SoftLDS<T> &S, uint32_t grp) {
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    GroupCtx G;
    double4 me;
    group_setup(A.src, A.gstart, A.sys_of, grp, G, me);
    const SysF P = A.sysf[G.sys];
    const SoftConst<T> Q(P);
    const T sx = (T)(me.x - G.c[0]);
    const T sy = (T)(me.y - G.c[1]);
    const T sz = (T)(me.z - G.c[2]);
    const double R2sq = P.R2sq;
    const T eps2 = Q.eps2;
    const T u2skip = Q.R2 * Q.R2 * (T)(1.0 + 0x1p-18);

    Acc<T> acc = {{0, 0, 0}, {0, 0, 0}, 0, 0};
    uint32_t n_pc = 0, n_far = 0, n_near = 0;
    int top = 1, npc = 0, nfr = 0, nnr = 0;
    uint32_t avail = 1, ftot = 0, ntot = 0;
    if (lane == 0) {
        S.sfirst[0] = G.sys;
        S.scnt[0] = 1;
    }
    __syncthreads();

    while (avail > 0) {
        const int want = step_width(top, avail);
        uint32_t id = take_items(S.sfirst, S.scnt, top, want, S.scan);
        avail -= (uint32_t)want;
        const bool have = lane < want;

        bool acc_c = false, leaf = false, opn = false, nr = false, sep = false;
        uint32_t first = 0, count = 0, child = 0, nch = 0;
        double ncom[3] = {0.0, 0.0, 0.0}, nM = 0.0, rb2 = 0.0, D2 = 0.0;
        if (have) {
            const Node nd = A.node[id];
            double D1 = dist2(gap_pt(G.lo[0], G.hi[0], nd.com[0]),
                              gap_pt(G.lo[1], G.hi[1], nd.com[1]),
                              gap_pt(G.lo[2], G.hi[2], nd.com[2]));
            D2 = dist2(gap_box(G.lo[0], G.hi[0], nd.blo[0], nd.blo[0] + nd.l),
                       gap_box(G.lo[1], G.hi[1], nd.blo[1], nd.blo[1] + nd.l),
                       gap_box(G.lo[2], G.hi[2], nd.blo[2], nd.blo[2] + nd.l));
            sep = HYBRID ? (D2 >= R2sq) : (D2 > 0.0);
            nch = nd.meta & 255u;
            rb2 = nd.rb2;
            acc_c = (D1 >= rb2) && sep;
            first = nd.first;
            count = nd.count;
            child = nd.child;
            for (int a = 0; a < 3; a++) ncom[a] = nd.com[a];
            nM = nd.M;
        }
        if (MINS) {
            // the paper's group rule: a cell is measured by its nearest sink,
            // min_i |u_i - COM|^2, never below the box distance D1, so the box
            // test above settles acceptances early; the others are decided
            // here, by all lanes together (sink positions are broadcast)
            const bool need = have && !acc_c && sep;
            if (__ballot(need)) {
                // the sinks' positions, read back as LDS broadcasts: the
                // particle tiles are free during a walk step
                static_assert(sizeof(S.tile) >= 3 * 64 * sizeof(double), "sink copy fits the tiles");
                double *sp = reinterpret_cast<double *>(&S.tile[0][0]);
                sp[lane] = me.x;
                sp[64 + lane] = me.y;
                sp[128 + lane] = me.z;
                __syncthreads();
                double Dm = INFINITY;
                for (int k = 0; k < G.ns; k++) {
                    const double dx = ncom[0] - sp[k], dy = ncom[1] - sp[64 + k],
                                 dz = ncom[2] - sp[128 + k];
                    Dm = fmin(Dm, fma(dz, dz, fma(dy, dy, dx * dx)));
                }
                if (need) acc_c = Dm >= rb2;
            }
        }
        leaf = have && !acc_c && nch == 0;
        opn = have && !acc_c && nch != 0;
        nr = HYBRID && leaf && (D2 < R2sq);
        vec4_t<T> pcs = make_vec4((T)0, (T)0, (T)0, (T)0);
        if (acc_c)
            pcs = make_vec4((T)(ncom[0] - G.c[0]), (T)(ncom[1] - G.c[1]), (T)(ncom[2] - G.c[2]),
                            (T)nM);
        const bool fr = leaf && !nr;
        if (over_capacity(A.status, npc + __popcll(__ballot(acc_c)) > kPC ||
                                        nfr + __popcll(__ballot(fr)) > kRQ ||
                                        nnr + __popcll(__ballot(nr)) > kRQ ||
                                        top + __popcll(__ballot(opn)) > kStk))
            break;
        // accepted cells -> particle-cell sources
        uint64_t m = __ballot(acc_c);
        if (acc_c) S.pc[npc + __popcll(m & lt)] = pcs;
        npc += __popcll(m);
        n_pc += __popcll(m);
        // rejected leaves -> far / near particle ranges
        m = __ballot(fr);
        if (fr) {
            int o = nfr + __popcll(m & lt);
            S.ffirst[o] = first;
            S.fcnt[o] = count;
        }
        nfr += __popcll(m);
        uint32_t cf = wave_sum(fr ? count : 0u);
        ftot += cf;
        n_far += cf;
        if (HYBRID) {
            m = __ballot(nr);
            if (nr) {
                int o = nnr + __popcll(m & lt);
                S.nfirst[o] = first;
                S.ncnt[o] = count;
            }
            nnr += __popcll(m);
            uint32_t cn = wave_sum(nr ? count : 0u);
            ntot += cn;
            n_near += cn;
        }
        // opened cells -> push their child ranges
        m = __ballot(opn);
        if (opn) {
            int o = top + __popcll(m & lt);
            S.sfirst[o] = child;
            S.scnt[o] = nch;
        }
        top += __popcll(m);
        avail += wave_sum(opn ? nch : 0u);
        HT_CHECK(top <= kStk && npc < kPC && nfr < kRQ && nnr < kRQ);
        __syncthreads();

        while (npc >= 64) {
            eval_far<POT, 64, T>(S.pc + (npc - 64), 64, sx, sy, sz, eps2, acc);
            npc -= 64;
        }
        // full particle tiles, double-buffered: the gather of the next tile
        // is in flight while the current one is evaluated
        if (ftot >= 64) {
            double4 q = A.src[take_items(S.ffirst, S.fcnt, nfr, 64, S.scan)];
            ftot -= 64;
            int buf = 0;
            for (;;) {
                S.tile[buf][lane] = rel_src<T>(q, G);
                __syncthreads();
                const bool more = ftot >= 64;
                if (more) {
                    q = A.src[take_items(S.ffirst, S.fcnt, nfr, 64, S.scan)];
                    ftot -= 64;
                }
                eval_far<POT, 64, T>(S.tile[buf], 64, sx, sy, sz, eps2, acc);
                if (!more) break;
                buf ^= 1;
            }
            __syncthreads();
        }
        if (HYBRID && ntot >= 64) {
            double4 q = A.src[take_items(S.nfirst, S.ncnt, nnr, 64, S.scan)];
            ntot -= 64;
            int buf = 0;
            for (;;) {
                S.tile[buf][lane] = rel_src<T>(q, G);
                __syncthreads();
                const bool more = ntot >= 64;
                if (more) {
                    q = A.src[take_items(S.nfirst, S.ncnt, nnr, 64, S.scan)];
                    ntot -= 64;
                }
                eval_near<POT, T>(S.tile[buf], 64, sx, sy, sz, eps2, Q.R2, Q.invdR, u2skip,
                                  acc);
                if (!more) break;
                buf ^= 1;
            }
            __syncthreads();
        }
    }
    // partial tiles
    if (npc > 0) eval_far<POT, 0, T>(S.pc, npc, sx, sy, sz, eps2, acc);
    if (ftot > 0) {
        int want = (int)ftot;
        uint32_t pi = take_items(S.ffirst, S.fcnt, nfr, want, S.scan);
        if (lane < want) S.tile[0][lane] = rel_src<T>(A.src[pi], G);
        __syncthreads();
        eval_far<POT, 0, T>(S.tile[0], want, sx, sy, sz, eps2, acc);
        __syncthreads();
    }
    if (HYBRID && ntot > 0) {
        int want = (int)ntot;
        uint32_t pi = take_items(S.nfirst, S.ncnt, nnr, want, S.scan);
        if (lane < want) S.tile[0][lane] = rel_src<T>(A.src[pi], G);
        __syncthreads();
        eval_near<POT, T>(S.tile[0], want, sx, sy, sz, eps2, Q.R2, Q.invdR, u2skip, acc);
        __syncthreads();
    }

    if (G.act) {
        const int64_t i = G.b0 + lane;
        const int64_t n = A.n;
        A.acc[i] = (float)(Q.G * (acc.a[0] - acc.c[0]));
        A.acc[n + i] = (float)(Q.G * (acc.a[1] - acc.c[1]));
        A.acc[2 * n + i] = (float)(Q.G * (acc.a[2] - acc.c[2]));
        if (POT) {
            // the sink itself was summed once among its own leaf's particles
            kahan(acc.p, acc.pc, (T)me.w * rsqrt_t(eps2));
            A.pot[i] = (float)(Q.G * (acc.p - acc.pc));
        }
    }
    if (A.wsoft && G.act) {
        // work measure for the next dispatch order: a near entry costs about
        // two far ones
        const uint64_t w = (uint64_t)n_pc + n_far + 2ull * n_near;
        A.wsoft[G.b0 + lane] = w > 0xffffffffull ? 0xffffffffu : (uint32_t)w;
    }
    if (lane == 0) {
        if (A.gcount) {
            A.gcount[grp] = n_pc;
            A.gcount[A.n + grp] = n_far;
            A.gcount[2 * A.n + grp] = n_near;
        }
        unsigned long long ent = (unsigned long long)n_pc + n_far + n_near;
        atomicAdd(&A.tally[tally_slot()], (unsigned long long)G.ns * ent);
    }
}

template <bool HYBRID, bool POT, bool MINS, typename T>
__global__ __launch_bounds__(64) void k_soft(ForceArgs A) {
    __shared__ SoftLDS<T> S;
    const uint32_t ng = *A.ng;
    for (uint32_t idx = blockIdx.x; idx < ng; idx += gridDim.x) {
        const uint32_t pos = sched_group(idx, ng);
        const uint32_t grp = A.order ? A.order[pos] : pos;
        HT_CHECK(grp < ng);
        HT_CHECK(A.gstart[grp + 1] > A.gstart[grp] && A.gstart[grp + 1] - A.gstart[grp] <= 64);
        soft_group<HYBRID, POT, MINS, T>(A, S, grp);
    }
}

template <bool MINS, typename T>
void launch_soft_t(const ForceArgs &A, bool hybrid, bool pot, dim3 grid, hipStream_t s) {
    dim3 block(64);
    if (hybrid) {
        if (pot) hipLaunchKernelGGL((k_soft<true, true, MINS, T>), grid, block, 0, s, A);
        else hipLaunchKernelGGL((k_soft<true, false, MINS, T>), grid, block, 0, s, A);
    } else {
        if (pot) hipLaunchKernelGGL((k_soft<false, true, MINS, T>), grid, block, 0, s, A);
        else hipLaunchKernelGGL((k_soft<false, false, MINS, T>), grid, block, 0, s, A);
    }
}

void launch_soft(const ForceArgs &A, bool hybrid, bool pot, int precision, bool min_sinks,
                 int n_wg, hipStream_t s) {
    HT_CHECK(n_wg > 0 && n_wg % 8 == 0);
    const dim3 grid((unsigned)n_wg);
    if (min_sinks) {
        if (precision == 1) launch_soft_t<true, double>(A, hybrid, pot, grid, s);
        else launch_soft_t<true, float>(A, hybrid, pot, grid, s);
    } else {
        if (precision == 1) launch_soft_t<false, double>(A, hybrid, pot, grid, s);
        else launch_soft_t<false, float>(A, hybrid, pot, grid, s);
    }
}

// ---------------------------------------------------------------------------
// hard force
// ---------------------------------------------------------------------------
constexpr int kHardEnt = 472;      // walk stack and leaf batch share these entries
constexpr int kStage = 192;        // staged candidates: up to 127 waiting + one gather of 64

// 10176 bytes: 16 wavefronts of this kernel fit the 160 KiB of a CU.
struct HardLDS {
    // walk stack (child ranges) in entries [0, top), the batch of collected
    // leaves (particle ranges) in entries [kHardEnt - nl, kHardEnt)
    uint32_t efirst[kHardEnt], ecnt[kHardEnt];
    double4 tq[kStage];            // staged candidate: master x, y, z and mass
    uint32_t scan[64];
};

// Gather order of a batch of nl collected leaves (leaf k in entry
// kHardEnt - 1 - k).  Consumption position q reads leaf (q * p) mod nl, with
// p the integer nearest nl (1 - 1/phi) that is coprime to nl (a bijection).
// Consecutive gathers so draw leaves from all over the batch, which spreads
// the pairs accepted in one stage over the group's sinks instead of piling
// them onto the few sinks next to one leaf; the accepted-pair loop runs as
// many times as the busiest lane needs.
struct LeafOrder {
    uint32_t nl = 1, p = 1;
    float inv = 1.0f;

    __device__ static LeafOrder make(uint32_t nl) {
        LeafOrder O;
        O.nl = nl;
        uint32_t p = (uint32_t)(0.381966f * (float)nl + 0.5f);
        if (p < 1u) p = 1u;
        for (;; p++) {            // gcd(p, nl) == 1; p = nl - 1 always is
            uint32_t a = nl, b = p;
            while (b) {
                uint32_t t = a % b;
                a = b;
                b = t;
            }
            if (a == 1u) break;
        }
        O.p = p;
        O.inv = 1.0f / (float)nl;
        return O;
    }
    // (q * p) mod nl for q < nl <= kHardEnt: q * p < 2^18 is exact in FP32 and
    // the quotient estimate is off by at most one either way.
    __device__ int slot(int q) const {
        const uint32_t t = (uint32_t)q * p;
        const uint32_t k = (uint32_t)((float)t * inv);
        int r = (int)(t - k * nl);
        if (r < 0) r += (int)nl;
        if (r >= (int)nl) r -= (int)nl;
        return kHardEnt - 1 - r;
    }
};

// Pair tests of this lane's sink against 64 staged candidates (unrolled), or
// against `cnt` <= 64 of them in a counted loop when CNT == 0: bit s of the
// result is set iff candidate s lies strictly inside R2 by the exact FP64
// test.  The two 32-bit halves of the mask are built separately: with a
// 64-bit shift and OR per candidate the compiler keeps ORing zeros into the
// other half.
template <int CNT>
__device__ inline uint64_t pair_tests(const double4 *t, int cnt, double xi, double yi, double zi,
                                      double R2sq) {
    uint32_t half[2] = {0u, 0u};
    if (CNT == 64) {
#pragma unroll
        for (int h = 0; h < 2; h++) {
#pragma unroll
            for (int b = 0; b < 32; b++) {
                const double4 q = t[32 * h + b];
                double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                half[h] |= r2 < R2sq ? 1u << b : 0u;
            }
        }
    } else {
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int e = cnt - 32 * h < 32 ? cnt - 32 * h : 32;
            for (int b = 0; b < e; b++) {
                const double4 q = t[32 * h + b];
                double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                half[h] |= r2 < R2sq ? 1u << b : 0u;
            }
        }
    }
    return (uint64_t)half[1] << 32 | half[0];
}

// 1/sqrt(s) in FP64: FP32 hardware seed (relative error about 1e-7), one
// Newton step (error about 1e-14).
__device__ inline double rsqrt64(double s) {
    double y = (double)rsq((float)s);
    return y * fma(-0.5 * s, y * y, 1.5);
}

template <int MODE>
__device__ void hard_group(const ForceArgs &A, HardLDS &S, uint32_t grp) {
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    const uint32_t b0 = A.gstart[grp];
    const uint32_t sys = A.sys_of[b0];
    const int ns = (int)(A.gstart[grp + 1] - b0);
    const bool act = lane < ns;
    const SysF P = A.sysf[sys];
    const int64_t n = A.n;
    const uint32_t mi = act ? b0 + lane : b0;
    const double4 me = A.xm[mi];
    const double xi = me.x, yi = me.y, zi = me.z;
    // box of the sinks' master positions (wave-uniform); the node boxes are
    // in master coordinates too
    double blo[3], bhi[3];
    {
        const double p[3] = {xi, yi, zi};
        for (int a = 0; a < 3; a++) {
            blo[a] = uniform_f64(wave_min(p[a]));
            bhi[a] = uniform_f64(wave_max(p[a]));
        }
    }
    const double R2sq = P.R2sq;
    const double pad2 = A.frame[sys].R2pad2;
    const double eps2d = P.eps2d, R2 = P.R2d, invdR64 = P.invdR64;

    // Accepted pairs are summed in FP64: the neighbour sum cancels strongly
    // (neighbours surround the sink), so FP32 per-pair rounding would be
    // magnified; FP64 FMA issues at the FP32 rate on this chip.  The sink
    // itself passes the test (r = 0) and adds exactly zero force; it is
    // removed from the neighbour count at the end.
    double hx = 0.0, hy = 0.0, hz = 0.0;
    uint32_t ngb = 0, cand = 0, trips = 0;

    // Search reuse between builds.  Record (mode 1): the walk opens the nodes
    // within the widened radius R2rec and keeps, in the group's list, every
    // node it tests and does not open; the leaves among them within R2 are
    // collected now.  Those nodes' subtrees cover every leaf exactly once.
    // Replay (mode 2, later launches over the same tree, boxes refitted to
    // new positions): the walk starts from the kept nodes instead of the
    // root and tests them against the current boxes with R2 -- close leaves
    // are collected, close inner nodes opened -- so the collected leaves are
    // exactly those a walk from the root would collect.
    constexpr int mode = MODE;   // 0 walk from the root, 1 record, 2 replay
    const int64_t lbase = (int64_t)kListPerSink * b0;
    const uint32_t lcap = kListPerSink * (uint32_t)ns;
    uint32_t elen = 0, epos = 0, hl = 0;
    bool from_root = true;
    if constexpr (mode == 2) {
        const uint32_t L = A.hlen[grp];
        if (L != kNoList) {
            elen = L;
            from_root = false;
        }
    }
    constexpr bool record = mode == 1;
    const double padw2 = record ? A.frame[sys].R2rec2 : pad2;   // opening radius
    int top = from_root ? 1 : 0, nl = 0, nr = 0, nst = 0;
    uint32_t avail = from_root ? 1u : 0u, tot = 0;
    if (lane == 0 && from_root) {
        S.efirst[0] = sys;
        S.ecnt[0] = 1;
    }
    __syncthreads();

    // tests and accepted-pair forces for the top `cnt` (<= 128) staged
    // candidates: full stages of 128 (during the walk) with the unrolled
    // tests, the rest (the final drain) with counted loops, whose code the
    // compiler does not reorder into 64 live compare masks
    auto eval_top = [&](int cnt, bool full) {
        const int base = nst - cnt;
        uint64_t m0, m1 = 0;
        if (full) {
            m0 = pair_tests<64>(S.tq + base, 64, xi, yi, zi, R2sq);
            m1 = pair_tests<64>(S.tq + base + 64, 64, xi, yi, zi, R2sq);
        } else {
            m0 = pair_tests<0>(S.tq + base, cnt < 64 ? cnt : 64, xi, yi, zi, R2sq);
            if (cnt > 64) m1 = pair_tests<0>(S.tq + base + 64, cnt - 64, xi, yi, zi, R2sq);
        }
        if (!act) m0 = m1 = 0;
        const uint32_t hits = (uint32_t)(__popcll(m0) + __popcll(m1));
        ngb += hits;
        if (A.cost) trips += wave_max_u32(hits);   // trips of the pair loop below
        int off = 0;
        while (m0 | m1) {
            // bits of the high word move down once the low word is spent
            const bool sw = m0 == 0;
            m0 = sw ? m1 : m0;
            m1 = sw ? 0 : m1;
            off = sw ? 64 : off;
            const int s = off + (int)__builtin_ctzll(m0);
            m0 &= m0 - 1;
            const double4 q = S.tq[base + s];
            double dx = q.x - xi, dy = q.y - yi, dz = q.z - zi;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            double ri = rsqrt64(r2 + eps2d);
            double r = r2 * rsqrt64(fmax(r2, 1e-30));   // the sink itself: r = 0
            double K = K_of64(r, R2, invdR64);
            double f = q.w * K * (ri * ri * ri);
            hx = fma(f, dx, hx);
            hy = fma(f, dy, hy);
            hz = fma(f, dz, hz);
        }
        cand += (uint32_t)cnt;
        nst -= cnt;
    };

    // Gathers of candidate particles from the batch of leaves, in two halves
    // so that the loads of one gather are in flight while staged pairs are
    // evaluated: issue() takes up to 64 particles and starts their loads,
    // finish() keeps those within R2 (plus slack) of the sink box.
    LeafOrder order;
    uint32_t g_pi = 0;
    int g_want = 0;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    float gm = 0.0f;
    auto issue = [&](int want) {
        g_pi = take_items(S.efirst, S.ecnt, nr, want, S.scan, order);
        g_want = want;
        if (lane < want) {
            const double4 q = A.xm[g_pi];
            gx = q.x;
            gy = q.y;
            gz = q.z;
            gm = (float)q.w;
        }
        tot -= (uint32_t)want;
    };
    auto finish = [&]() {
        bool keep = false;
        if (lane < g_want) {
            double D = dist2(gap_pt(blo[0], bhi[0], gx), gap_pt(blo[1], bhi[1], gy),
                             gap_pt(blo[2], bhi[2], gz));
            keep = D < pad2;
        }
        uint64_t m = __ballot(keep);
        if (keep) S.tq[nst + __popcll(m & lt)] = make_double4(gx, gy, gz, (double)gm);
        nst += __popcll(m);
        g_want = 0;
        __syncthreads();
    };
    // gathers every particle of the collected leaves in the batch's order,
    // overlapping each gather's loads with evaluation; empties the batch
    auto drain_batch = [&]() {
        order = LeafOrder::make((uint32_t)nl);
        nr = nl;
        bool pending = false;
        for (;;) {
            if (pending) finish();
            pending = tot > 0;
            if (pending) issue(tot < 64u ? (int)tot : 64);
            if (nst >= 128) eval_top(128, true);
            if (!pending) break;
        }
        HT_CHECK(nr == 0);
        nl = 0;
    };

    // The walk collects leaves into the batch until the shared entries run
    // short, then the batch is gathered.  Nodes come from the stack of pushed
    // child ranges first, then from the replayed list.
    while (avail > 0 || epos < elen) {
        // one entry beyond the depth-first reserve is kept for a leaf
        int room = kHardEnt - kStkReserve - 1 - top - nl;
        if (nl > 0 && room < 64) {
            drain_batch();
            room = kHardEnt - kStkReserve - 1 - top;
        }
        uint32_t id = 0;
        int want;
        if (mode != 2 || avail > 0) {
            want = avail < 64u ? (int)avail : 64;
            if (want > room) want = room > 1 ? room : 1;
            id = take_items(S.efirst, S.ecnt, top, want, S.scan);
            avail -= (uint32_t)want;
        } else {
            want = elen - epos < 64u ? (int)(elen - epos) : 64;
            if (want > room) want = room > 1 ? room : 1;
            if (lane < want) id = A.hlist[lbase + epos + (uint32_t)lane];
            epos += (uint32_t)want;
        }
        // each node taken adds at most one entry (a pushed range or a leaf)
        if (over_capacity(A.status, top + nl + want > kHardEnt)) break;
        const bool have = lane < want;
        bool leaf = false, opn = false, keep = false;
        uint32_t first = 0, count = 0, child = 0, nch = 0;
        if (have) {
            const double4 *bx = (const double4 *)A.aabb + 2 * (int64_t)id;
            const double4 bl = bx[0], bh = bx[1];
            double D2 = dist2(gap_box(blo[0], bhi[0], bl.x, bh.x),
                              gap_box(blo[1], bhi[1], bl.y, bh.y),
                              gap_box(blo[2], bhi[2], bl.z, bh.z));
            const Node &nd = A.node[id];
            nch = nd.meta & 255u;
            leaf = D2 < pad2 && nch == 0;
            opn = D2 < padw2 && nch != 0;
            keep = !opn;
            first = nd.first;
            count = nd.count;
            child = nd.child;
        }
        uint64_t m;
        if constexpr (record) {
            m = __ballot(keep);
            const uint32_t pos = hl + (uint32_t)__popcll(m & lt);
            if (keep && pos < lcap) A.hlist[lbase + pos] = id;
            hl += (uint32_t)__popcll(m);
        }
        m = __ballot(leaf);
        if (leaf) {
            int o = kHardEnt - 1 - (nl + __popcll(m & lt));
            S.efirst[o] = first;
            S.ecnt[o] = count;
        }
        nl += __popcll(m);
        tot += wave_sum(leaf ? count : 0u);
        m = __ballot(opn);
        if (opn) {
            int o = top + __popcll(m & lt);
            S.efirst[o] = child;
            S.ecnt[o] = nch;
        }
        top += __popcll(m);
        avail += wave_sum(opn ? nch : 0u);
        HT_CHECK(top + nl <= kHardEnt && nst < kStage);
        __syncthreads();
    }
    if (nl > 0) drain_batch();
    while (nst > 0) eval_top(nst < 128 ? nst : 128, false);

    if (act) {
        const int64_t i = b0 + lane;
        ngb -= 1u;    // the sink itself
        A.acc[i] = (float)(P.Gd * hx);
        A.acc[n + i] = (float)(P.Gd * hy);
        A.acc[2 * n + i] = (float)(P.Gd * hz);
        if (A.ngb) A.ngb[i] = (int32_t)ngb;
    }
    uint32_t ngb_sum = wave_sum(act ? ngb : 0u);
    // work measure for the dispatch order: a pair-loop trip costs about seven
    // candidate tests
    if (A.cost && lane == 0) A.cost[grp] = cand + 7u * trips;
    if constexpr (record) {
        if (lane == 0) A.hlen[grp] = hl <= lcap ? hl : kNoList;
    }
    if (lane == 0) {
        atomicAdd(&A.tally[tally_slot() + 1], (unsigned long long)ns * cand);
        atomicAdd(&A.tally[tally_slot() + 2], (unsigned long long)ngb_sum);
    }
}

template <int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_hard(ForceArgs A) {
    __shared__ HardLDS S;
    const uint32_t ng = *A.ng;
    for (uint32_t idx = blockIdx.x; idx < ng; idx += gridDim.x) {
        const uint32_t pos = sched_group(idx, ng);
        const uint32_t grp = A.order ? A.order[pos] : pos;
        HT_CHECK(grp < ng);
        hard_group<MODE>(A, S, grp);
    }
}

void launch_hard(const ForceArgs &A, int n_wg, hipStream_t s) {
    HT_CHECK(n_wg > 0 && n_wg % 8 == 0);
    const dim3 grid((unsigned)n_wg), block(64);
    if (A.hmode == 1) hipLaunchKernelGGL(k_hard<1>, grid, block, 0, s, A);
    else if (A.hmode == 2) hipLaunchKernelGGL(k_hard<2>, grid, block, 0, s, A);
    else hipLaunchKernelGGL(k_hard<0>, grid, block, 0, s, A);
}

}  // namespace htree
