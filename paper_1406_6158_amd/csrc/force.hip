// force.hip -- soft (tree) and hard (neighbour) force kernels for gfx950.
//
// Soft force (section II.B walk, grouped sinks of section III.A.2, split of
// section II.C).  One wavefront serves one group of 64 consecutive
// key-ordered sinks, one sink per lane.  The walk is wide depth-first: each
// step pops up to 64 nodes from an LDS stack, one per lane, and tests them in
// FP64 against the group's bounding box:
//   D1 = dist^2(box_g, COM),  D2 = dist^2(box_g, cell box)
//   accepted iff D1 >= r_b^2 and (hybrid ? D2 >= R2^2 : D2 > 0).
// Accepted cells become particle-cell sources, rejected leaves particle
// sources ("near", weighted by 1 - K, iff hybrid and D2 < R2^2), other nodes
// push their (contiguous) children.  Sources are staged in LDS as FP32
// offsets from the group centre plus mass; every 64 of them all lanes run the
// interaction loop, FP32 per tile, tiles merged with compensated (Kahan)
// summation.  No list leaves the chip.
//
// The stack stays bounded: a step that pops p nodes grows the stack by at
// most 7p, so p is capped to keep a reserve of 160 entries; once the reserve
// is reached the walk proceeds one node at a time, depth first, which adds at
// most 7 entries per level on the current path (7 x 21 = 147).
//
// Hard force (section II.C, eq. 10): per group, a walk that opens every node
// whose box lies within R2 (plus rounding slack) of the group box collects
// candidate leaves; each candidate pair is decided by the exact FP64 test
// fma(dz,dz, fma(dy,dy, dx*dx)) < R2^2 on the master positions, and accepted
// pairs add K(r) times the softened pair force in FP32.
#include "htree_dev.h"

#include <math.h>

namespace htree {

constexpr int kStk = 1024;
constexpr int kStkReserve = 160;
constexpr int kPC = 128;
constexpr int kRQ = 128;

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ inline void kahan(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

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
__device__ inline float one_minus_K(float r, float R2f, float invdR) {
    float Y = (R2f - r) * invdR;
    Y = fminf(fmaxf(Y, 0.0f), 1.0f);
    float w = fmaf(-Y, Y, 1.0f);
    float t = fmaf(fmaf(6.0f, w, -15.0f), w, 10.0f);
    return t * (w * w * w);
}
__device__ inline float K_of(float r, float R2f, float invdR) {
    float Y = (R2f - r) * invdR;
    Y = fminf(fmaxf(Y, 0.0f), 1.0f);
    float s = Y * Y;
    float t = fmaf(fmaf(6.0f, s, -15.0f), s, 10.0f);
    return t * (s * s * s);
}

// Group setup shared by both walks.
struct GroupCtx {
    int64_t b0;
    int ns;
    bool act;
    double lo[3], hi[3], c[3];
};

__device__ inline void group_setup(const double4 *src, int64_t n, int g, int64_t grp,
                                   GroupCtx &G, double4 &me) {
    const int lane = threadIdx.x;
    G.b0 = grp * g;
    int64_t e0 = G.b0 + g < n ? G.b0 + g : n;
    G.ns = (int)(e0 - G.b0);
    G.act = lane < G.ns;
    me = src[G.act ? G.b0 + lane : G.b0];
    double p[3] = {me.x, me.y, me.z};
    for (int a = 0; a < 3; a++) {
        G.lo[a] = wave_min(p[a]);
        G.hi[a] = wave_max(p[a]);
        G.c[a] = 0.5 * (G.lo[a] + G.hi[a]);
    }
}

// ---------------------------------------------------------------------------
// interaction loops
// ---------------------------------------------------------------------------
struct Acc {
    float a[3], c[3];   // running sums and Kahan compensations
    float p, pc;
};

template <bool POT, int CNT>
__device__ inline void eval_far(const float4 *t, int cnt, float sx, float sy, float sz, float eps2,
                                Acc &A) {
    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
    const int nloop = CNT > 0 ? CNT : cnt;
#pragma unroll 8
    for (int j = 0; j < nloop; j++) {
        float4 q = t[j];
        float dx = q.x - sx, dy = q.y - sy, dz = q.z - sz;
        float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
        float ri = rsq(r2);
        float mr = q.w * ri;
        float f = mr * (ri * ri);
        ax = fmaf(f, dx, ax);
        ay = fmaf(f, dy, ay);
        az = fmaf(f, dz, az);
        if (POT) ph -= mr;
    }
    kahan(A.a[0], A.c[0], ax);
    kahan(A.a[1], A.c[1], ay);
    kahan(A.a[2], A.c[2], az);
    if (POT) kahan(A.p, A.pc, ph);
}

template <bool POT>
__device__ inline void eval_near(const float4 *t, int cnt, float sx, float sy, float sz,
                                 float eps2, float R2f, float invdR, Acc &A) {
    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
#pragma unroll 4
    for (int j = 0; j < cnt; j++) {
        float4 q = t[j];
        float dx = q.x - sx, dy = q.y - sy, dz = q.z - sz;
        float u2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        float ri = rsq(u2 + eps2);
        float mr = q.w * ri;
        float w = one_minus_K(fsqrt(u2), R2f, invdR);
        float f = mr * (ri * ri) * w;
        ax = fmaf(f, dx, ax);
        ay = fmaf(f, dy, ay);
        az = fmaf(f, dz, az);
        if (POT) ph -= mr;
    }
    kahan(A.a[0], A.c[0], ax);
    kahan(A.a[1], A.c[1], ay);
    kahan(A.a[2], A.c[2], az);
    if (POT) kahan(A.p, A.pc, ph);
}

// Takes `want` particles from the top of a leaf-range stack (first[], cnt[],
// nr ranges), consuming each range from its end, and returns for this lane
// (lane < want) the sorted particle index.  Updates nr and the partially
// consumed range.  All lanes must call it.
__device__ inline uint32_t take_particles(uint32_t *first, uint32_t *cnt, int &nr, int want,
                                          uint32_t *scan) {
    const int lane = threadIdx.x;
    int r = nr < 64 ? nr : 64;
    uint32_t ck = 0, fk = 0;
    if (lane < r) {
        ck = cnt[nr - 1 - lane];
        fk = first[nr - 1 - lane];
    }
    uint32_t inc = wave_incl_scan(ck);
    scan[lane] = inc;
    __syncthreads();
    uint32_t pidx = 0;
    if (lane < want) {
        int lo = 0, hi = r - 1;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (scan[mid] > (uint32_t)lane) hi = mid; else lo = mid + 1;
        }
        uint32_t prev = lo ? scan[lo - 1] : 0u;
        uint32_t f = first[nr - 1 - lo], c = cnt[nr - 1 - lo];
        pidx = f + c - 1u - ((uint32_t)lane - prev);
    }
    uint64_t full = __ballot(lane < r && inc <= (uint32_t)want);
    int nfull = __popcll(full);
    uint32_t used = nfull ? __shfl(inc, nfull - 1) : 0u;
    __syncthreads();
    if (lane == 0 && (uint32_t)want > used) cnt[nr - 1 - nfull] -= (uint32_t)want - used;
    nr -= nfull;
    __syncthreads();
    return pidx;
}

// ---------------------------------------------------------------------------
// soft force
// ---------------------------------------------------------------------------
struct SoftLDS {
    uint32_t stk[kStk];
    float4 pc[kPC];
    float4 tile[64];
    uint32_t ffirst[kRQ], fcnt[kRQ];
    uint32_t nfirst[kRQ], ncnt[kRQ];
    uint32_t scan[64];
};

template <bool HYBRID, bool POT>
__global__ __launch_bounds__(64) void k_soft(ForceArgs A) {
    __shared__ SoftLDS S;
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt();
    const int64_t grp = xcd_item(blockIdx.x, A.n_groups);
    GroupCtx G;
    double4 me;
    group_setup(A.src, A.n, A.g, grp, G, me);
    const float sx = (float)(me.x - G.c[0]);
    const float sy = (float)(me.y - G.c[1]);
    const float sz = (float)(me.z - G.c[2]);
    const double R2sq = A.R2sq;
    const float eps2 = A.eps2;

    Acc acc = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, 0.f, 0.f};
    uint32_t n_pc = 0, n_far = 0, n_near = 0;
    int top = 1, npc = 0, nfr = 0, nnr = 0;
    uint32_t ftot = 0, ntot = 0;
    if (lane == 0) S.stk[0] = 0;
    __syncthreads();

    while (top > 0) {
        int p = top < 64 ? top : 64;
        int pmax = (kStk - kStkReserve - top) / 7;
        if (p > pmax) p = pmax > 1 ? pmax : 1;
        const bool have = lane < p;
        uint32_t id = have ? S.stk[top - p + lane] : 0u;
        top -= p;
        __syncthreads();

        bool acc_c = false, leaf = false, opn = false, nr = false;
        uint32_t first = 0, count = 0, child = 0, nch = 0;
        float4 pcs = make_float4(0.f, 0.f, 0.f, 0.f);
        if (have) {
            const Node nd = A.node[id];
            double D1 = dist2(gap_pt(G.lo[0], G.hi[0], nd.com[0]),
                              gap_pt(G.lo[1], G.hi[1], nd.com[1]),
                              gap_pt(G.lo[2], G.hi[2], nd.com[2]));
            double D2 = dist2(gap_box(G.lo[0], G.hi[0], nd.blo[0], nd.blo[0] + nd.l),
                              gap_box(G.lo[1], G.hi[1], nd.blo[1], nd.blo[1] + nd.l),
                              gap_box(G.lo[2], G.hi[2], nd.blo[2], nd.blo[2] + nd.l));
            bool sep = HYBRID ? (D2 >= R2sq) : (D2 > 0.0);
            nch = nd.meta & 255u;
            acc_c = (D1 >= nd.rb2) && sep;
            leaf = !acc_c && nch == 0;
            opn = !acc_c && nch != 0;
            nr = HYBRID && leaf && (D2 < R2sq);
            first = nd.first;
            count = nd.count;
            child = nd.child;
            if (acc_c)
                pcs = make_float4((float)(nd.com[0] - G.c[0]), (float)(nd.com[1] - G.c[1]),
                                  (float)(nd.com[2] - G.c[2]), (float)nd.M);
        }
        // accepted cells -> particle-cell sources
        uint64_t m = __ballot(acc_c);
        if (acc_c) S.pc[npc + __popcll(m & lt)] = pcs;
        npc += __popcll(m);
        n_pc += __popcll(m);
        // rejected leaves -> far / near particle ranges
        const bool fr = leaf && !nr;
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
        // opened cells -> push children
        uint32_t k = opn ? nch : 0u;
        uint32_t inc = wave_incl_scan(k);
        if (opn) {
            uint32_t b = (uint32_t)top + inc - k;
            for (uint32_t j = 0; j < k; j++) S.stk[b + j] = child + j;
        }
        top += (int)__shfl(inc, 63);
        __syncthreads();

        while (npc >= 64) {
            eval_far<POT, 64>(S.pc + (npc - 64), 64, sx, sy, sz, eps2, acc);
            npc -= 64;
        }
        while (ftot >= 64) {
            uint32_t pi = take_particles(S.ffirst, S.fcnt, nfr, 64, S.scan);
            double4 q = A.src[pi];
            S.tile[lane] = make_float4((float)(q.x - G.c[0]), (float)(q.y - G.c[1]),
                                       (float)(q.z - G.c[2]), (float)q.w);
            __syncthreads();
            eval_far<POT, 64>(S.tile, 64, sx, sy, sz, eps2, acc);
            __syncthreads();
            ftot -= 64;
        }
        if (HYBRID) {
            while (ntot >= 64) {
                uint32_t pi = take_particles(S.nfirst, S.ncnt, nnr, 64, S.scan);
                double4 q = A.src[pi];
                S.tile[lane] = make_float4((float)(q.x - G.c[0]), (float)(q.y - G.c[1]),
                                           (float)(q.z - G.c[2]), (float)q.w);
                __syncthreads();
                eval_near<POT>(S.tile, 64, sx, sy, sz, eps2, A.R2f, A.invdR, acc);
                __syncthreads();
                ntot -= 64;
            }
        }
    }
    // partial tiles
    if (npc > 0) eval_far<POT, 0>(S.pc, npc, sx, sy, sz, eps2, acc);
    if (ftot > 0) {
        int want = (int)ftot;
        uint32_t pi = take_particles(S.ffirst, S.fcnt, nfr, want, S.scan);
        if (lane < want) {
            double4 q = A.src[pi];
            S.tile[lane] = make_float4((float)(q.x - G.c[0]), (float)(q.y - G.c[1]),
                                       (float)(q.z - G.c[2]), (float)q.w);
        }
        __syncthreads();
        eval_far<POT, 0>(S.tile, want, sx, sy, sz, eps2, acc);
        __syncthreads();
    }
    if (HYBRID && ntot > 0) {
        int want = (int)ntot;
        uint32_t pi = take_particles(S.nfirst, S.ncnt, nnr, want, S.scan);
        if (lane < want) {
            double4 q = A.src[pi];
            S.tile[lane] = make_float4((float)(q.x - G.c[0]), (float)(q.y - G.c[1]),
                                       (float)(q.z - G.c[2]), (float)q.w);
        }
        __syncthreads();
        eval_near<POT>(S.tile, want, sx, sy, sz, eps2, A.R2f, A.invdR, acc);
    }

    if (G.act) {
        const int64_t i = G.b0 + lane;
        const int64_t n = A.n;
        A.acc[i] = A.G * (acc.a[0] - acc.c[0]);
        A.acc[n + i] = A.G * (acc.a[1] - acc.c[1]);
        A.acc[2 * n + i] = A.G * (acc.a[2] - acc.c[2]);
        if (POT) {
            // the sink itself was summed once among its own leaf's particles
            kahan(acc.p, acc.pc, (float)me.w * rsq(eps2));
            A.pot[i] = A.G * (acc.p - acc.pc);
        }
    }
    if (lane == 0) {
        if (A.gcount) {
            A.gcount[grp] = n_pc;
            A.gcount[A.n_groups + grp] = n_far;
            A.gcount[2 * A.n_groups + grp] = n_near;
        }
        unsigned long long ent = (unsigned long long)n_pc + n_far + n_near;
        atomicAdd(&A.tally[0], (unsigned long long)G.ns * ent);
    }
}

void launch_soft(const ForceArgs &A, bool hybrid, bool pot, hipStream_t s) {
    dim3 grid((unsigned)A.n_groups), block(64);
    if (hybrid) {
        if (pot) hipLaunchKernelGGL((k_soft<true, true>), grid, block, 0, s, A);
        else hipLaunchKernelGGL((k_soft<true, false>), grid, block, 0, s, A);
    } else {
        if (pot) hipLaunchKernelGGL((k_soft<false, true>), grid, block, 0, s, A);
        else hipLaunchKernelGGL((k_soft<false, false>), grid, block, 0, s, A);
    }
}

// ---------------------------------------------------------------------------
// hard force
// ---------------------------------------------------------------------------
struct HardLDS {
    uint32_t stk[kStk];
    double tx[64], ty[64], tz[64];
    float tm[64];
    uint32_t ti[64];
    uint32_t rfirst[kRQ], rcnt[kRQ];
    uint32_t scan[64];
};

__global__ __launch_bounds__(64) void k_hard(ForceArgs A) {
    __shared__ HardLDS S;
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt();
    const int64_t grp = xcd_item(blockIdx.x, A.n_groups);
    GroupCtx G;
    double4 me;
    group_setup(A.src, A.n, A.g, grp, G, me);
    const int64_t n = A.n;
    const int64_t mi = G.act ? G.b0 + lane : G.b0;
    const double xi = A.x[mi], yi = A.x[n + mi], zi = A.x[2 * n + mi];
    const uint32_t myidx = (uint32_t)mi;
    const double R2sq = A.R2sq;
    const double pad2 = A.frame->R2pad2;
    const float eps2 = A.eps2, R2f = A.R2f, invdR = A.invdR;

    Acc acc = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, 0.f, 0.f};
    uint32_t ngb = 0, cand = 0;
    int top = 1, nr = 0;
    uint32_t tot = 0;
    if (lane == 0) S.stk[0] = 0;
    __syncthreads();

    auto eval_tile = [&](int cnt) {
        uint64_t mask = 0;
        for (int s = 0; s < cnt; s++) {
            double dx = S.tx[s] - xi, dy = S.ty[s] - yi, dz = S.tz[s] - zi;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            bool in = (r2 < R2sq) && (S.ti[s] != myidx);
            mask |= (uint64_t)in << s;
        }
        if (!G.act) mask = 0;
        ngb += __popcll(mask);
        float hx = 0.f, hy = 0.f, hz = 0.f;
        while (mask) {
            int s = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            double dx = S.tx[s] - xi, dy = S.ty[s] - yi, dz = S.tz[s] - zi;
            double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            float fx = (float)dx, fy = (float)dy, fz = (float)dz;
            float u2 = (float)r2;
            float ri = rsq(u2 + eps2);
            float K = K_of(fsqrt(u2), R2f, invdR);
            float f = S.tm[s] * K * (ri * ri * ri);
            hx = fmaf(f, fx, hx);
            hy = fmaf(f, fy, hy);
            hz = fmaf(f, fz, hz);
        }
        kahan(acc.a[0], acc.c[0], hx);
        kahan(acc.a[1], acc.c[1], hy);
        kahan(acc.a[2], acc.c[2], hz);
    };
    auto fill_tile = [&](int want) {
        uint32_t pi = take_particles(S.rfirst, S.rcnt, nr, want, S.scan);
        if (lane < want) {
            S.tx[lane] = A.x[pi];
            S.ty[lane] = A.x[n + pi];
            S.tz[lane] = A.x[2 * n + pi];
            S.tm[lane] = (float)A.src[pi].w;
            S.ti[lane] = pi;
        }
        __syncthreads();
    };

    while (top > 0) {
        int p = top < 64 ? top : 64;
        int pmax = (kStk - kStkReserve - top) / 7;
        if (p > pmax) p = pmax > 1 ? pmax : 1;
        const bool have = lane < p;
        uint32_t id = have ? S.stk[top - p + lane] : 0u;
        top -= p;
        __syncthreads();
        bool leaf = false, opn = false;
        uint32_t first = 0, count = 0, child = 0, nch = 0;
        if (have) {
            const Node nd = A.node[id];
            double D2 = dist2(gap_box(G.lo[0], G.hi[0], nd.blo[0], nd.blo[0] + nd.l),
                              gap_box(G.lo[1], G.hi[1], nd.blo[1], nd.blo[1] + nd.l),
                              gap_box(G.lo[2], G.hi[2], nd.blo[2], nd.blo[2] + nd.l));
            nch = nd.meta & 255u;
            bool close = D2 < pad2;
            leaf = close && nch == 0;
            opn = close && nch != 0;
            first = nd.first;
            count = nd.count;
            child = nd.child;
        }
        uint64_t m = __ballot(leaf);
        if (leaf) {
            int o = nr + __popcll(m & lt);
            S.rfirst[o] = first;
            S.rcnt[o] = count;
        }
        nr += __popcll(m);
        tot += wave_sum(leaf ? count : 0u);
        uint32_t k = opn ? nch : 0u;
        uint32_t inc = wave_incl_scan(k);
        if (opn) {
            uint32_t b = (uint32_t)top + inc - k;
            for (uint32_t j = 0; j < k; j++) S.stk[b + j] = child + j;
        }
        top += (int)__shfl(inc, 63);
        __syncthreads();
        while (tot >= 64) {
            fill_tile(64);
            eval_tile(64);
            cand += 64;
            __syncthreads();
            tot -= 64;
        }
    }
    if (tot > 0) {
        fill_tile((int)tot);
        eval_tile((int)tot);
        cand += tot;
    }
    if (G.act) {
        const int64_t i = G.b0 + lane;
        A.acc[i] = A.G * (acc.a[0] - acc.c[0]);
        A.acc[n + i] = A.G * (acc.a[1] - acc.c[1]);
        A.acc[2 * n + i] = A.G * (acc.a[2] - acc.c[2]);
        if (A.ngb) A.ngb[i] = (int32_t)ngb;
    }
    uint32_t ngb_sum = wave_sum(G.act ? ngb : 0u);
    if (lane == 0) {
        atomicAdd(&A.tally[1], (unsigned long long)G.ns * cand);
        atomicAdd(&A.tally[2], (unsigned long long)ngb_sum);
    }
}

void launch_hard(const ForceArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_hard, dim3((unsigned)A.n_groups), dim3(64), 0, s, A);
}

}  // namespace htree
