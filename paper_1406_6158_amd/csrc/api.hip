// api.hip -- host implementation of the C ABI declared in include/htree.h:
// parameter validation, workspace carving, stream-ordered orchestration of
// the build / force / integrator kernels, status and counters.  A context
// holds S >= 1 systems (htree_create is the case S = 1).
#include "../../include/htree.h"
#include "htree_dev.h"
#include "internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

using namespace htree;

namespace {

thread_local std::string g_err;

htree_status fail(htree_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
htree_status fail(htree_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace

htree_status htree::set_error(htree_status code, const char *msg) {
    g_err = msg;
    return code;
}

namespace {

#define HIP_OK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(HTREE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

constexpr int64_t kMaxN = (int64_t)1 << 27;      // particles per context
constexpr int32_t kMaxSys = 1 << 16;             // systems per context
constexpr int64_t kChunk = 1 << 12;              // bounding-box chunk (one block each)

bool is_fin(double v) { return isfinite(v) != 0; }

htree_status validate_one(const htree_params *p, int64_t n) {
    if (n < 1 || n > kMaxN) return fail(HTREE_EINVAL, "n = %lld outside [1, 2^27]", (long long)n);
    if (!is_fin(p->G) || p->G <= 0) return fail(HTREE_EINVAL, "G must be finite and > 0");
    if (!is_fin(p->eps) || p->eps < 1e-15)
        return fail(HTREE_EINVAL, "eps must be finite and >= 1e-15");
    if (!is_fin(p->theta) || p->theta < 0) return fail(HTREE_EINVAL, "theta must be >= 0");
    if (p->hybrid != 0 && p->hybrid != 1) return fail(HTREE_EINVAL, "hybrid must be 0 or 1");
    if (p->hybrid && !(is_fin(p->R1) && is_fin(p->R2) && p->R1 > 0 && p->R2 > p->R1))
        return fail(HTREE_EINVAL, "hybrid mode needs 0 < R1 < R2");
    if (!is_fin(p->dt_soft)) return fail(HTREE_EINVAL, "dt_soft must be finite");
    if (p->n_sub < 1 || p->n_sub > 1024) return fail(HTREE_EINVAL, "n_sub must be in [1, 1024]");
    if (p->n_crit < 1 || p->n_crit > 4096) return fail(HTREE_EINVAL, "n_crit must be in [1, 4096]");
    if (p->group_size < 1 || p->group_size > 64)
        return fail(HTREE_EINVAL, "group_size must be in [1, 64]");
    if (p->precision != 0 && p->precision != 1)
        return fail(HTREE_EINVAL, "precision must be 0 (FP32) or 1 (FP64 interactions)");
    if (p->flags & ~(HTREE_F_POT | HTREE_F_TIMING | HTREE_F_REUSE))
        return fail(HTREE_EINVAL, "unknown flags");
    if (p->group_cell < 1 || p->group_cell > 4096)
        return fail(HTREE_EINVAL, "group_cell must be in [1, 4096]");
    if (p->group_mac != 0 && p->group_mac != 1)
        return fail(HTREE_EINVAL, "group_mac must be 0 (box distance) or 1 (minimum over sinks)");
    if (!is_fin(p->a_err) || p->a_err < 0) return fail(HTREE_EINVAL, "a_err must be >= 0");
    return HTREE_OK;
}

// Every system is checked; the integrator and layout settings must agree.
htree_status validate(const htree_params *p, const int64_t *n, int32_t S) {
    if (!p || !n) return fail(HTREE_EINVAL, "params or sizes are NULL");
    if (S < 1 || S > kMaxSys) return fail(HTREE_EINVAL, "system count %d outside [1, 65536]", S);
    int64_t tot = 0;
    for (int32_t s = 0; s < S; s++) {
        htree_status st = validate_one(&p[s], n[s]);
        if (st) return st;
        const htree_params &a = p[0], &b = p[s];
        if (b.dt_soft != a.dt_soft || b.n_sub != a.n_sub || b.hybrid != a.hybrid ||
            b.precision != a.precision || b.flags != a.flags || b.group_mac != a.group_mac)
            return fail(HTREE_EINVAL, "system %d: dt_soft, n_sub, hybrid, precision, flags and "
                                      "group_mac must equal those of system 0", s);
        tot += n[s];
    }
    if (tot > kMaxN) return fail(HTREE_EINVAL, "total particles %lld exceed 2^27", (long long)tot);
    return HTREE_OK;
}

// Upper bound on the node count: at each of the levels 0..20 the internal
// nodes hold disjoint sets of >= n_crit particles, and leaves are disjoint and
// non-empty.
int64_t max_nodes(int64_t n, int n_crit) { return 1 + 21 * (n / n_crit) + n; }

struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += sizeof(T) * (size_t)(count > 0 ? count : 1);
        return p;
    }
};

}  // namespace

struct htree_ctx {
    htree_params p;                    // shared settings (system 0)
    std::vector<htree_params> ps;      // per system
    std::vector<int64_t> ns;           // particles per system
    int32_t S = 1;
    int64_t n = 0, ng = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    BuildBufs B;
    float *tmp3 = nullptr;             // [3][n] caller-order input staged in key order
    float *pot = nullptr;              // [n] key order
    int32_t *ngb = nullptr;            // [n] key order
    uint32_t *gcount = nullptr;        // [3][n] list sizes per group (first ng used)
    unsigned long long *tally = nullptr;      // [kTallySlots][kTallyStride] slots
    unsigned long long *tally_sum = nullptr;  // [4] their totals (launch_tally_fold)
    int n_wg = 0;                      // force kernel grid
    std::vector<Sys> h_sys;            // host copies of the static tables, kept
    std::vector<SysF> h_sysf;          // alive until the asynchronous upload is
    std::vector<uint2> h_chunk;        // surely done (the context's lifetime)
    bool tree = false, moments = false, have_soft = false, have_hard = false;
    bool boxes = false;                // node boxes fit the current positions (hard walk)
    bool hard_order = false;           // B.horder holds an order for the current hard groups
    bool hard_lists = false;           // B.hlist holds recorded searches over the current tree
    bool topo = false;                 // a tree was built since the last set_state
    bool forces_current = false;
    bool timing = false;
    bool on_scratch = false;           // carved from the library's static scratch
    std::vector<hipEvent_t> ev[3];     // per phase: start/end pairs since the last stats
    int ev_n[3] = {0, 0, 0};
    int calls[3] = {0, 0, 0};
};

namespace {

int64_t chunk_count(const std::vector<int64_t> &ns) {
    int64_t c = 0;
    for (int64_t n : ns) c += (n + kChunk - 1) / kChunk;
    return c;
}

void carve(Carver &C, htree_ctx *c) {
    const int64_t n = c->n;
    const int32_t S = c->S;
    BuildBufs &B = c->B;
    B.n = n;
    B.S = S;
    B.sysbits = 0;
    while ((1 << B.sysbits) < S) B.sysbits++;
    B.max_n_crit = 0;
    B.abs_mac = false;
    for (int32_t s = 0; s < S; s++) B.abs_mac |= c->ps[s].a_err > 0.0;
    B.nchunks = chunk_count(c->ns);
    B.nnmax = 0;
    for (int32_t s = 0; s < S; s++) {
        B.nnmax += max_nodes(c->ns[s], c->ps[s].n_crit);
        if (c->ps[s].n_crit > B.max_n_crit) B.max_n_crit = c->ps[s].n_crit;
    }
    const int64_t nnmax = B.nnmax;
    B.sys = C.take<Sys>(S);
    B.sysf = C.take<SysF>(S);
    B.sys_of = C.take<uint32_t>(n);
    B.chunk = C.take<uint2>(B.nchunks);
    for (int k = 0; k < 2; k++) {
        B.x[k] = C.take<double>(3 * n);
        B.v[k] = C.take<float>(3 * n);
        B.m[k] = C.take<float>(n);
        B.perm[k] = C.take<uint32_t>(n);
        B.as[k] = C.take<float>(3 * n);
        B.ah[k] = C.take<float>(3 * n);
        B.key[k] = C.take<uint64_t>(n);
        B.idx[k] = C.take<uint32_t>(n);
    }
    if (S > 1) {
        B.skey[0] = C.take<uint32_t>(n);
        B.skey[1] = C.take<uint32_t>(n);
        B.ktmp = C.take<uint64_t>(n);
    } else {
        B.skey[0] = B.skey[1] = nullptr;
        B.ktmp = nullptr;
    }
    B.src = C.take<double4>(n);
    // the largest sorts: nodes (nnmax) and the dispatch keys of both group kinds (2n)
    const int64_t nsort = nnmax > 2 * n ? nnmax : 2 * n;
    const int64_t hb = 256 * sort_blocks(nsort);
    B.hist = C.take<uint32_t>(hb + (int64_t)scan_partials(hb));
    B.bbox_part = C.take<double>(6 * B.nchunks);
    B.frame = C.take<Frame>(S);
    B.status = C.take<uint32_t>(4);
    B.cpl = C.take<int8_t>(n);
    B.leaflev = C.take<int8_t>(n);
    B.nstart = C.take<uint32_t>(n + 1);
    // partials of the largest scan: n + 1 flags, the sort histograms, and
    // (absolute MAC) the nnmax + 1 chunk counts of the b_max pass
    int64_t sp = (int64_t)scan_partials(n + 1);
    int64_t sp2 = (int64_t)scan_partials(256 * sort_blocks(nsort));
    int64_t sp3 = B.abs_mac ? (int64_t)scan_partials(nnmax + 1) : 0;
    if (sp2 > sp) sp = sp2;
    if (sp3 > sp) sp = sp3;
    B.scan_part = C.take<uint32_t>(sp);
    B.nn = C.take<uint32_t>(4);
    B.pre_key = C.take<uint32_t>(nnmax);
    B.pre_val = C.take<uint32_t>(nnmax);
    B.lvl_key2 = C.take<uint32_t>(nnmax > n ? nnmax : n);
    B.bfs2pre = C.take<uint32_t>(nnmax);
    B.pre2bfs = C.take<uint32_t>(nnmax);
    B.pre_first = C.take<uint32_t>(nnmax);
    B.pre_count = C.take<uint32_t>(nnmax);
    if (B.sysbits + 5 > 8) {
        B.ptmp_k = C.take<uint32_t>(nnmax);
        B.ptmp_v = C.take<uint32_t>(nnmax);
    } else {
        B.ptmp_k = B.ptmp_v = nullptr;
    }
    B.node = C.take<Node>(nnmax);
    B.B2 = C.take<double>(B.abs_mac ? nnmax : 1);
    B.bmax = C.take<unsigned long long>(B.abs_mac ? nnmax : 1);
    B.bitems = C.take<uint32_t>(B.abs_mac ? nnmax + 1 : 1);
    B.S3 = C.take<double>(3 * nnmax);
    B.aabb = C.take<double>(8 * nnmax);
    B.xm = C.take<double4>(n);
    {
        int64_t m1, m2, m3;
        refit_sizes(n, &m1, &m2, &m3);
        B.cbox = C.take<double>(6 * (m1 + m2 + m3));
    }
    B.lstart = C.take<uint32_t>(kMaxLevel + 2);
    B.gstart = C.take<uint32_t>(n + 1);
    B.ng = C.take<uint32_t>(4);
    B.hgstart = C.take<uint32_t>(n + 1);
    B.nhg = C.take<uint32_t>(4);
    B.hcost = C.take<uint32_t>(2 * n);
    B.hkey = C.take<uint32_t>(2 * n);
    B.hval = C.take<uint32_t>(2 * n);
    B.horder = C.take<uint32_t>(n);
    B.hlist = C.take<uint32_t>((int64_t)kListPerSink * n);
    B.hlen = C.take<uint32_t>(n);
    B.ndisp = C.take<uint32_t>(4);
    c->tmp3 = C.take<float>(3 * n);
    c->pot = C.take<float>(n);
    c->ngb = C.take<int32_t>(n);
    c->gcount = C.take<uint32_t>(3 * n);
    for (int k = 0; k < 2; k++) {
        B.wsoft[k] = C.take<uint32_t>(n);
        B.whard[k] = C.take<uint32_t>(n);
    }
    B.sorder = C.take<uint32_t>(2 * n);
    c->tally = C.take<unsigned long long>(kTallySlots * kTallyStride);
    c->tally_sum = C.take<unsigned long long>(4);
}

void setup_sizes(htree_ctx *c, const htree_params *p, const int64_t *n, int32_t S) {
    c->S = S;
    c->ps.assign(p, p + S);
    c->ns.assign(n, n + S);
    c->p = p[0];
    c->n = 0;
    for (int32_t s = 0; s < S; s++) c->n += n[s];
}

size_t footprint(const htree_params *p, const int64_t *n, int32_t S) {
    htree_ctx tmp;
    setup_sizes(&tmp, p, n, S);
    Carver C{nullptr};
    carve(C, &tmp);
    return (C.off + 255) & ~(size_t)255;
}

// Host-side static tables, uploaded once at creation.
htree_status upload_tables(htree_ctx *c) {
    const int32_t S = c->S;
    std::vector<Sys> &sys = c->h_sys;
    std::vector<SysF> &sysf = c->h_sysf;
    std::vector<uint2> &chunks = c->h_chunk;
    sys.assign(S, Sys{});
    sysf.assign(S, SysF{});
    chunks.clear();
    uint32_t p0 = 0;
    for (int32_t s = 0; s < S; s++) {
        const htree_params &q = c->ps[s];
        Sys &y = sys[s];
        y.p0 = p0;
        y.p1 = p0 + (uint32_t)c->ns[s];
        y.c0 = (uint32_t)chunks.size();
        for (int64_t a = y.p0; a < y.p1; a += kChunk) {
            int64_t b = a + kChunk < y.p1 ? a + kChunk : y.p1;
            chunks.push_back(make_uint2((uint32_t)a, (uint32_t)b));
        }
        y.c1 = (uint32_t)chunks.size();
        y.n_crit = (uint32_t)q.n_crit;
        y.g = (uint32_t)q.group_size;
        y.gcell = (uint32_t)q.group_cell;
        y.invth2 = 1.0 / (q.theta * q.theta);
        y.aerr = q.a_err;
        y.G = q.G;
        y.R2 = q.hybrid ? q.R2 : 0.0;
        SysF &f = sysf[s];
        f.G = (float)q.G;
        f.eps2 = (float)(q.eps * q.eps);
        f.R2f = (float)q.R2;
        f.invdR = q.hybrid ? (float)(1.0 / (q.R2 - q.R1)) : 0.0f;
        f.R2sq = q.R2 * q.R2;
        f.Gd = q.G;
        f.eps2d = q.eps * q.eps;
        f.R2d = q.R2;
        f.invdR64 = q.hybrid ? 1.0 / (q.R2 - q.R1) : 0.0;
        p0 = y.p1;
    }
    BuildBufs &B = c->B;
    // stream-ordered: a context created while other work runs does not wait for it
    HIP_OK(hipMemcpyAsync(B.sys, sys.data(), sizeof(Sys) * S, hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(B.sysf, sysf.data(), sizeof(SysF) * S, hipMemcpyHostToDevice,
                          c->stream));
    HIP_OK(hipMemcpyAsync(B.chunk, chunks.data(), sizeof(uint2) * chunks.size(),
                          hipMemcpyHostToDevice, c->stream));
    launch_sys_of(B, c->stream);
    HIP_OK(hipGetLastError());
    return HTREE_OK;
}

ForceArgs force_args(htree_ctx *c) {
    ForceArgs A;
    const BuildBufs &B = c->B;
    A.node = B.node;
    A.gstart = B.gstart;
    A.ng = B.ng;
    A.sys_of = B.sys_of;
    A.sysf = B.sysf;
    A.src = B.src;
    A.aabb = B.aabb;
    A.xm = B.xm;
    A.nnmax = B.nnmax;
    A.frame = B.frame;
    A.order = nullptr;
    A.cost = nullptr;
    A.wsoft = nullptr;
    A.hlist = nullptr;
    A.hlen = nullptr;
    A.hmode = 0;
    A.n = c->n;
    A.acc = nullptr;
    A.pot = nullptr;
    A.ngb = nullptr;
    A.gcount = c->gcount;
    A.tally = c->tally;
    A.status = B.status;
    return A;
}

void ev_begin(htree_ctx *c, int k) {
    c->calls[k]++;
    if (!c->timing) return;
    std::vector<hipEvent_t> &v = c->ev[k];
    size_t need = 2 * (size_t)(c->ev_n[k] + 1);
    while (v.size() < need) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;
        v.push_back(e);
    }
    (void)hipEventRecord(v[2 * c->ev_n[k]], c->stream);
}
void ev_end(htree_ctx *c, int k) {
    if (!c->timing) return;
    std::vector<hipEvent_t> &v = c->ev[k];
    if (v.size() < 2 * (size_t)(c->ev_n[k] + 1)) return;
    (void)hipEventRecord(v[2 * c->ev_n[k] + 1], c->stream);
    c->ev_n[k]++;
}

// keep_acc: permute the kept accelerations too (not needed when both forces
// are computed right after the build).
htree_status do_build(htree_ctx *c, bool moments, bool keep_acc = true) {
    ev_begin(c, 0);
    launch_bbox_keys(c->B, c->stream);
    launch_sort(c->B, c->stream);
    launch_gather(c->B, keep_acc, c->stream);
    launch_topology(c->B, moments, c->stream);
    launch_groups(c->B, c->stream);
    launch_dispatch_orders(c->B, c->stream);
    ev_end(c, 0);
    HIP_OK(hipGetLastError());
    c->tree = true;
    c->boxes = true;
    c->hard_order = false;
    c->hard_lists = false;
    c->topo = true;
    c->moments = moments;
    return HTREE_OK;
}

// After a drift: the node boxes are recomputed from the drifted positions over
// the same tree (same sorted order, nodes and groups).  Enough for the hard
// force, whose walk needs only boxes that contain the particles; the soft
// force needs a full build.
htree_status do_refit(htree_ctx *c) {
    ev_begin(c, 0);
    launch_refit(c->B, c->stream);
    ev_end(c, 0);
    HIP_OK(hipGetLastError());
    c->boxes = true;
    return HTREE_OK;
}

htree_status do_soft(htree_ctx *c) {
    if (!c->tree || !c->moments) return fail(HTREE_ESTATE, "soft_force needs a current tree");
    ForceArgs A = force_args(c);
    A.acc = c->B.as[c->B.cur];
    const bool pot = (c->p.flags & HTREE_F_POT) != 0;
    A.pot = pot ? c->pot : nullptr;
    A.order = c->B.sorder;
    A.wsoft = c->B.wsoft[c->B.cur];
    ev_begin(c, 1);
    launch_soft(A, c->p.hybrid != 0, pot, c->p.precision, c->p.group_mac != 0, c->n_wg,
                c->stream);
    ev_end(c, 1);
    HIP_OK(hipGetLastError());
    c->have_soft = true;
    return HTREE_OK;
}

htree_status do_hard(htree_ctx *c) {
    if (!c->p.hybrid) return fail(HTREE_EINVAL, "hard_force needs hybrid mode");
    if (!c->boxes) return fail(HTREE_ESTATE, "hard_force needs a current tree");
    ForceArgs A = force_args(c);
    A.gstart = c->B.hgstart;   // the hard kernel's own groups
    A.ng = c->B.nhg;
    A.acc = c->B.ah[c->B.cur];
    A.ngb = c->ngb;
    // groups run heaviest first: the first launch over new groups by the
    // costs carried from the last build's groups, and it measures their own
    // costs, which order the later launches (after refits)
    A.order = c->B.horder;
    A.cost = c->hard_order ? nullptr : c->B.hcost;
    // with reuse, the first launch over a tree records each group's search
    // (widened by the skin); the launches after refits replay it against the
    // new boxes
    const bool reuse = (c->p.flags & HTREE_F_REUSE) != 0;
    A.hlist = c->B.hlist;
    A.hlen = c->B.hlen;
    A.hmode = !reuse ? 0 : c->hard_lists ? 2 : 1;
    ev_begin(c, 2);
    launch_hard(A, c->n_wg, c->stream);
    if (!c->hard_order) launch_hard_order(c->B, c->stream);
    ev_end(c, 2);
    c->hard_order = true;
    c->hard_lists = true;
    HIP_OK(hipGetLastError());
    c->have_hard = true;
    return HTREE_OK;
}

htree_status kick(htree_ctx *c, double ks, double kh, double dt_drift) {
    BuildBufs &B = c->B;
    const int k = B.cur;
    launch_kick_drift(B.x[k], B.xm, B.m[k], B.v[k], ks != 0.0 ? B.as[k] : nullptr, (float)ks,
                      kh != 0.0 ? B.ah[k] : nullptr, (float)kh, dt_drift, c->n, c->stream);
    HIP_OK(hipGetLastError());
    if (dt_drift != 0.0) c->tree = c->moments = c->boxes = c->forces_current = false;
    return HTREE_OK;
}

htree_status ensure_forces(htree_ctx *c) {
    if (c->forces_current) return HTREE_OK;
    htree_status st = do_build(c, true, false);
    if (st) return st;
    if ((st = do_soft(c))) return st;
    if (c->p.hybrid && (st = do_hard(c))) return st;
    c->forces_current = true;
    return HTREE_OK;
}

#define CTX_CHECK(c)                                                         \
    do {                                                                     \
        if (!(c)) return fail(HTREE_EINVAL, "context is NULL");             \
        HIP_OK(hipSetDevice((c)->device));                                   \
    } while (0)

}  // namespace

// ---------------------------------------------------------------------------
// Static scratch: the workspace of htree_create_static, for callers that
// cannot allocate device memory.  Each device holds its own copy until the
// process ends; one context at a time may use it.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = HTREE_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];      // device address of scratch, per device
bool g_scratch_held[kMaxDevices];      // a live context uses it

htree_status create_ctx(htree_ctx **out, const htree_params *p, const int64_t *n, int32_t S,
                        void *ws, size_t ws_bytes, void *stream);

}  // namespace

extern "C" {

void htree_default_params(htree_params *p) {
    if (!p) return;
    p->G = 1.0;
    p->eps = 0.01;
    p->theta = 0.5;
    p->R1 = 0.05;
    p->R2 = 0.1;
    p->dt_soft = 1.0 / 16.0;
    p->n_sub = 4;
    p->hybrid = 1;
    p->n_crit = 16;
    p->group_size = 64;
    p->precision = 0;
    p->flags = 0;
    p->group_cell = 16;
    p->group_mac = 0;
    p->a_err = 0.0;
}

size_t htree_batch_workspace_bytes(const htree_params *p, const int64_t *n, int32_t S) {
    if (validate(p, n, S) != HTREE_OK) return 0;
    return footprint(p, n, S);
}

size_t htree_workspace_bytes(const htree_params *p, int64_t n) {
    return htree_batch_workspace_bytes(p, &n, 1);
}

htree_status htree_batch_create(htree_ctx **out, const htree_params *p, const int64_t *n,
                                int32_t S, void *ws, size_t ws_bytes, void *stream) {
    return create_ctx(out, p, n, S, ws, ws_bytes, stream);
}

htree_status htree_create(htree_ctx **out, const htree_params *p, int64_t n, void *ws,
                          size_t ws_bytes, void *stream) {
    return htree_batch_create(out, p, &n, 1, ws, ws_bytes, stream);
}

htree_status htree_create_static(htree_ctx **out, const htree_params *p, int64_t n,
                                 void *stream) {
    if (!out) return fail(HTREE_EINVAL, "out is NULL");
    *out = nullptr;
    htree_status st = validate(p, &n, 1);
    if (st) return st;
    const size_t need = footprint(p, &n, 1);
    if (need > kScratchBytes)
        return fail(HTREE_ENOMEM,
                    "n = %lld needs %zu workspace bytes, more than the %zu of the static scratch",
                    (long long)n, need, kScratchBytes);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HTREE_EINVAL, "device %d out of range", dev);
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // the array's name is a host-side stand-in; its device address is
            // looked up once per device, with that device current
            void *ptr = nullptr;
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(HTREE_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                            hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
        if (g_scratch_held[dev])
            return fail(HTREE_ESTATE, "the static scratch of device %d is held by another "
                        "context; destroy that one first", dev);
        g_scratch_held[dev] = true;
        ws = g_scratch_ptr[dev];
    }
    st = create_ctx(out, p, &n, 1, ws, kScratchBytes, stream);
    if (st) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_scratch_held[dev] = false;
        return st;
    }
    (*out)->on_scratch = true;
    return HTREE_OK;
}

}  // extern "C"

namespace {

htree_status create_ctx(htree_ctx **out, const htree_params *p, const int64_t *n, int32_t S,
                        void *ws, size_t ws_bytes, void *stream) {
    if (!out) return fail(HTREE_EINVAL, "out is NULL");
    *out = nullptr;
    htree_status st = validate(p, n, S);
    if (st) return st;
    size_t need = footprint(p, n, S);
    if (!ws) return fail(HTREE_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255u) != 0) return fail(HTREE_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < need)
        return fail(HTREE_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    htree_ctx *c = new htree_ctx();
    setup_sizes(c, p, n, S);
    c->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&c->device);
    int cus = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e != hipSuccess) {
        delete c;
        return fail(HTREE_EDEVICE, "device query: %s", hipGetErrorString(e));
    }
    // force kernels: one one-wavefront workgroup per group for groups of 16
    // or more sinks on average (typical groups hold about 45), at least one
    // per slot of the chip (16 per CU), a multiple of 8; workgroups past the
    // group count exit at once, groups past the grid are taken in a
    // grid-stride loop
    {
        int64_t want = c->n / 16 + c->S + 64;
        const int64_t fill = (int64_t)(cus > 0 ? cus : 256) * 16;
        if (want < fill) want = fill;
        if (want > ((int64_t)1 << 30)) want = (int64_t)1 << 30;
        want = (want + 7) & ~(int64_t)7;
        c->n_wg = (int)want;
    }
    Carver C{(char *)ws};
    carve(C, c);
    c->B.cur = 0;
    c->timing = (p[0].flags & HTREE_F_TIMING) != 0;
    launch_zero_u32(c->B.status, 4, c->stream);
    launch_zero_u32(c->B.nn, 4, c->stream);
    launch_zero_u32((uint32_t *)c->tally, 2 * kTallySlots * kTallyStride, c->stream);
    if ((st = upload_tables(c))) {
        delete c;
        return st;
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        delete c;
        return fail(HTREE_EDEVICE, "launch: %s", hipGetErrorString(e));
    }
    *out = c;
    return HTREE_OK;
}

}  // namespace

extern "C" {

int32_t htree_system_count(htree_ctx *c) { return c ? c->S : -1; }

htree_status htree_set_state(htree_ctx *c, const double *d_x, const float *d_v, const float *d_m) {
    CTX_CHECK(c);
    return htree::ctx_set_state(c, d_x, c->n, d_v, d_m);
}

htree_status htree_build_tree(htree_ctx *c) {
    CTX_CHECK(c);
    c->forces_current = false;
    return do_build(c, true);
}

htree_status htree_soft_force(htree_ctx *c, float *d_acc, float *d_pot) {
    CTX_CHECK(c);
    if (d_pot && !(c->p.flags & HTREE_F_POT))
        return fail(HTREE_EINVAL, "d_pot given but the context lacks HTREE_F_POT");
    htree_status st = do_soft(c);
    if (st) return st;
    const BuildBufs &B = c->B;
    if (d_acc) launch_scatter3(B.as[B.cur], B.perm[B.cur], d_acc, c->n, c->stream);
    if (d_pot) launch_scatter1f(c->pot, B.perm[B.cur], d_pot, c->n, c->stream);
    HIP_OK(hipGetLastError());
    return HTREE_OK;
}

htree_status htree_hard_force(htree_ctx *c, float *d_acc, int32_t *d_ngb) {
    CTX_CHECK(c);
    htree_status st = do_hard(c);
    if (st) return st;
    const BuildBufs &B = c->B;
    if (d_acc) launch_scatter3(B.ah[B.cur], B.perm[B.cur], d_acc, c->n, c->stream);
    if (d_ngb) launch_scatter1i(c->ngb, B.perm[B.cur], d_ngb, c->n, c->stream);
    HIP_OK(hipGetLastError());
    return HTREE_OK;
}

htree_status htree_kick_drift(htree_ctx *c, double dt_kick, const float *d_acc, double dt_drift) {
    CTX_CHECK(c);
    if (!is_fin(dt_kick) || !is_fin(dt_drift)) return fail(HTREE_EINVAL, "non-finite dt");
    BuildBufs &B = c->B;
    const int k = B.cur;
    if (d_acc) {
        launch_gather3(d_acc, B.perm[k], c->tmp3, c->n, c->stream);
        launch_kick_drift(B.x[k], B.xm, B.m[k], B.v[k], c->tmp3, (float)dt_kick, nullptr, 0.f,
                          dt_drift, c->n, c->stream);
    } else {
        if (!c->have_soft && !c->have_hard)
            return fail(HTREE_ESTATE, "no kept accelerations to kick with");
        launch_kick_drift(B.x[k], B.xm, B.m[k], B.v[k], c->have_soft ? B.as[k] : nullptr,
                          (float)dt_kick, c->have_hard ? B.ah[k] : nullptr, (float)dt_kick,
                          dt_drift, c->n, c->stream);
    }
    HIP_OK(hipGetLastError());
    if (dt_drift != 0.0) c->tree = c->moments = c->boxes = c->forces_current = false;
    return HTREE_OK;
}

htree_status htree_refit(htree_ctx *c) {
    CTX_CHECK(c);
    if (!c->topo) return fail(HTREE_ESTATE, "refit needs a built tree");
    return do_refit(c);
}

htree_status htree_step(htree_ctx *c, int32_t n_soft) {
    CTX_CHECK(c);
    if (n_soft < 0) return fail(HTREE_EINVAL, "n_soft_steps must be >= 0");
    htree_status st = ensure_forces(c);
    if (st) return st;
    const double dts = c->p.dt_soft;
    // The closing half-kicks of a (sub)step and the opening half-kicks of the
    // next use the same forces, so they are applied together, with the next
    // drift, in one launch; the closing kicks of the call's last substep are
    // applied at its end.
    double pend_s = 0.0, pend_h = 0.0;
    for (int32_t s = 0; s < n_soft; s++) {
        if (!c->p.hybrid) {
            if ((st = kick(c, pend_s + 0.5 * dts, 0.0, dts))) return st;
            if ((st = do_build(c, true, false))) return st;
            if ((st = do_soft(c))) return st;
            pend_s = 0.5 * dts;
            continue;
        }
        const int nsub = c->p.n_sub;
        const double dth = dts / nsub;
        for (int h = 0; h < nsub; h++) {
            // opening kicks (soft half-kick on the first substep), the
            // pending closing kicks, and the drift
            if ((st = kick(c, pend_s + (h == 0 ? 0.5 * dts : 0.0), pend_h + 0.5 * dth, dth)))
                return st;
            // a full build where the soft force needs it, a refit of the
            // node boxes on the other substeps
            const bool last = h == nsub - 1;
            if ((st = last ? do_build(c, true, false) : do_refit(c))) return st;
            if (last && (st = do_soft(c))) return st;
            if ((st = do_hard(c))) return st;
            pend_s = last ? 0.5 * dts : 0.0;
            pend_h = 0.5 * dth;
        }
    }
    if (pend_s != 0.0 || pend_h != 0.0) {
        if ((st = kick(c, pend_s, pend_h, 0.0))) return st;
    }
    c->forces_current = true;
    return HTREE_OK;
}

htree_status htree_get_state(htree_ctx *c, double *d_x, float *d_v) {
    CTX_CHECK(c);
    const BuildBufs &B = c->B;
    if (d_x) launch_scatter_x(B.x[B.cur], B.perm[B.cur], d_x, c->n, c->stream);
    if (d_v) launch_scatter3(B.v[B.cur], B.perm[B.cur], d_v, c->n, c->stream);
    HIP_OK(hipGetLastError());
    return HTREE_OK;
}

htree_status htree_sync(htree_ctx *c) {
    CTX_CHECK(c);
    HIP_OK(hipStreamSynchronize(c->stream));
    uint32_t st = 0;
    HIP_OK(hipMemcpy(&st, c->B.status, sizeof st, hipMemcpyDeviceToHost));
    return htree::status_code(st);
}

htree_status htree_stats(htree_ctx *c, htree_counters *out) {
    CTX_CHECK(c);
    if (!out) return fail(HTREE_EINVAL, "out is NULL");
    HIP_OK(hipStreamSynchronize(c->stream));
    unsigned long long t[4];
    uint32_t nn = 0, ng = 0;
    launch_tally_fold(c->tally, c->tally_sum, c->stream);
    HIP_OK(hipMemcpyAsync(t, c->tally_sum, sizeof t, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(&nn, c->B.nn, sizeof nn, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&ng, c->B.ng, sizeof ng, hipMemcpyDeviceToHost));
    c->ng = ng;
    memset(out, 0, sizeof *out);
    out->n = c->n;
    out->n_groups = ng;
    out->n_nodes = nn;
    out->soft_interactions = (int64_t)t[0];
    out->hard_candidates = (int64_t)t[1];
    out->hard_pairs = (int64_t)t[2];
    if (c->have_soft) {
        const int64_t n = c->n;
        std::vector<uint32_t> h(3 * (size_t)ng + 1);
        for (int k = 0; k < 3; k++)
            HIP_OK(hipMemcpy(h.data() + k * (size_t)ng, c->gcount + k * n, sizeof(uint32_t) * ng,
                             hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < ng; k++) {
            out->soft_cells += h[k];
            out->soft_far += h[ng + k];
            out->soft_near += h[2 * ng + k];
        }
    }
    float *dst[3] = {&out->ms_build, &out->ms_soft, &out->ms_hard};
    for (int k = 0; k < 3; k++) {
        float tot = 0.f;
        for (int j = 0; j < c->ev_n[k]; j++) {
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, c->ev[k][2 * j], c->ev[k][2 * j + 1]));
            tot += ms;
        }
        *dst[k] = tot;
        c->ev_n[k] = 0;
    }
    out->calls_build = c->calls[0];
    out->calls_soft = c->calls[1];
    out->calls_hard = c->calls[2];
    c->calls[0] = c->calls[1] = c->calls[2] = 0;
    launch_zero_u32((uint32_t *)c->tally, 2 * kTallySlots * kTallyStride, c->stream);
    HIP_OK(hipGetLastError());
    return HTREE_OK;
}

htree_status htree_group_counts(htree_ctx *c, int32_t *n_cells, int32_t *n_far, int32_t *n_near) {
    CTX_CHECK(c);
    if (!c->have_soft) return fail(HTREE_ESTATE, "no soft_force has run");
    HIP_OK(hipStreamSynchronize(c->stream));
    uint32_t ng = 0;
    HIP_OK(hipMemcpy(&ng, c->B.ng, sizeof ng, hipMemcpyDeviceToHost));
    int32_t *dst[3] = {n_cells, n_far, n_near};
    for (int k = 0; k < 3; k++)
        if (dst[k])
            HIP_OK(hipMemcpy(dst[k], c->gcount + k * c->n, sizeof(int32_t) * ng,
                             hipMemcpyDeviceToHost));
    return HTREE_OK;
}

htree_status htree_export_keys(htree_ctx *c, uint64_t *keys, int32_t *perm, double *frame4) {
    CTX_CHECK(c);
    if (!c->tree) return fail(HTREE_ESTATE, "no current tree");
    HIP_OK(hipStreamSynchronize(c->stream));
    const BuildBufs &B = c->B;
    if (keys) HIP_OK(hipMemcpy(keys, B.key[0], sizeof(uint64_t) * c->n, hipMemcpyDeviceToHost));
    if (perm)
        HIP_OK(hipMemcpy(perm, B.perm[B.cur], sizeof(int32_t) * c->n, hipMemcpyDeviceToHost));
    if (frame4) {
        std::vector<Frame> F(c->S);
        HIP_OK(hipMemcpy(F.data(), B.frame, sizeof(Frame) * c->S, hipMemcpyDeviceToHost));
        for (int32_t s = 0; s < c->S; s++) {
            frame4[4 * s + 0] = F[s].lo[0];
            frame4[4 * s + 1] = F[s].lo[1];
            frame4[4 * s + 2] = F[s].lo[2];
            frame4[4 * s + 3] = F[s].side;
        }
    }
    return HTREE_OK;
}

int64_t htree_node_count(htree_ctx *c) {
    if (!c) return -1;
    if (hipSetDevice(c->device) != hipSuccess) return -1;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
    uint32_t nn = 0;
    if (hipMemcpy(&nn, c->B.nn, sizeof nn, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return nn;
}

htree_status htree_export_nodes(htree_ctx *c, int32_t *level, int32_t *first, int32_t *count,
                                double *mass, double *com) {
    CTX_CHECK(c);
    if (!c->tree) return fail(HTREE_ESTATE, "no current tree");
    int64_t nn = htree_node_count(c);
    if (nn < 0) return fail(HTREE_EDEVICE, "cannot read the node count");
    std::vector<Node> h(nn > 0 ? nn : 1);
    HIP_OK(hipMemcpy(h.data(), c->B.node, sizeof(Node) * nn, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < nn; k++) {
        if (level) level[k] = (int32_t)(h[k].meta >> 8);
        if (first) first[k] = (int32_t)h[k].first;
        if (count) count[k] = (int32_t)h[k].count;
        if (mass) mass[k] = h[k].M;
        if (com)
            for (int a = 0; a < 3; a++) com[a * nn + k] = h[k].com[a];
    }
    return HTREE_OK;
}

htree_status htree_export_node_boxes(htree_ctx *c, double *lo, double *hi) {
    CTX_CHECK(c);
    if (!c->topo || !c->boxes) return fail(HTREE_ESTATE, "no node boxes for the current positions");
    int64_t nn = htree_node_count(c);
    if (nn < 0) return fail(HTREE_EDEVICE, "cannot read the node count");
    std::vector<double> h(8 * (nn > 0 ? nn : 1));
    HIP_OK(hipMemcpy(h.data(), c->B.aabb, sizeof(double) * 8 * nn, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < nn; k++)
        for (int a = 0; a < 3; a++) {
            if (lo) lo[a * nn + k] = h[8 * k + a];
            if (hi) hi[a * nn + k] = h[8 * k + 4 + a];
        }
    return HTREE_OK;
}

htree_status htree_export_node_mac(htree_ctx *c, double *B2, double *bmax2, double *rb2) {
    CTX_CHECK(c);
    if (!c->tree) return fail(HTREE_ESTATE, "no current tree");
    HIP_OK(hipStreamSynchronize(c->stream));
    uint32_t nn = 0;
    HIP_OK(hipMemcpy(&nn, c->B.nn, sizeof nn, hipMemcpyDeviceToHost));
    if (B2 || bmax2) {
        if (c->B.abs_mac) {
            std::vector<unsigned long long> bits(nn);
            if (B2) HIP_OK(hipMemcpy(B2, c->B.B2, sizeof(double) * nn, hipMemcpyDeviceToHost));
            if (bmax2) {
                HIP_OK(hipMemcpy(bits.data(), c->B.bmax, sizeof(unsigned long long) * nn,
                                 hipMemcpyDeviceToHost));
                memcpy(bmax2, bits.data(), sizeof(double) * nn);
            }
        } else {
            if (B2) memset(B2, 0, sizeof(double) * nn);
            if (bmax2) memset(bmax2, 0, sizeof(double) * nn);
        }
    }
    if (rb2) {
        std::vector<Node> h(nn);
        HIP_OK(hipMemcpy(h.data(), c->B.node, sizeof(Node) * nn, hipMemcpyDeviceToHost));
        for (uint32_t k = 0; k < nn; k++) rb2[k] = h[k].rb2;
    }
    return HTREE_OK;
}

int64_t htree_group_count(htree_ctx *c) {
    if (!c || !c->tree) return -1;
    if (hipSetDevice(c->device) != hipSuccess) return -1;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
    uint32_t ng = 0;
    if (hipMemcpy(&ng, c->B.ng, sizeof ng, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return ng;
}

htree_status htree_export_groups(htree_ctx *c, int32_t *starts) {
    CTX_CHECK(c);
    if (!c->tree) return fail(HTREE_ESTATE, "no current tree");
    int64_t ng = htree_group_count(c);
    if (ng < 0) return fail(HTREE_EDEVICE, "cannot read the group count");
    if (starts)
        HIP_OK(hipMemcpy(starts, c->B.gstart, sizeof(int32_t) * (ng + 1), hipMemcpyDeviceToHost));
    return HTREE_OK;
}

const char *htree_last_error(void) { return g_err.c_str(); }

void htree_destroy(htree_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    for (int k = 0; k < 3; k++)
        for (hipEvent_t e : c->ev[k]) (void)hipEventDestroy(e);
    if (c->on_scratch) {
        // the next context on this device's scratch must not overwrite it
        // while this one's work is still running
        (void)hipStreamSynchronize(c->stream);
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_scratch_held[c->device] = false;
    }
    delete c;
}

}  // extern "C"

htree_status htree::ctx_set_state(htree_ctx *c, const double *d_x, int64_t ldx, const float *d_v,
                                  const float *d_m) {
    if (!d_x || !d_m) return fail(HTREE_EINVAL, "x and m are required");
    if (ldx < c->n) return fail(HTREE_EINVAL, "x row stride %lld < n", (long long)ldx);
    BuildBufs &B = c->B;
    B.cur = 0;
    launch_set_state(d_x, ldx, d_v, d_m, B.x[0], B.v[0], B.m[0], B.perm[0], c->n, c->stream);
    launch_zero_u32((uint32_t *)B.as[0], 3 * c->n, c->stream);
    launch_zero_u32((uint32_t *)B.ah[0], 3 * c->n, c->stream);
    launch_zero_u32(B.wsoft[0], c->n, c->stream);
    launch_zero_u32(B.whard[0], c->n, c->stream);
    HIP_OK(hipGetLastError());
    c->tree = c->moments = c->boxes = c->have_soft = c->have_hard = c->forces_current = false;
    c->hard_order = false;
    c->topo = false;
    return HTREE_OK;
}

htree_status htree::ctx_report_async(htree_ctx *c, CtxReport *dst) {
    // the status word and the interaction tallies, copied in stream order
    HIP_OK(hipMemcpyAsync(&dst->status, c->B.status, sizeof(uint32_t), hipMemcpyDeviceToHost,
                          c->stream));
    launch_tally_fold(c->tally, c->tally_sum, c->stream);
    HIP_OK(hipMemcpyAsync(dst->tally, c->tally_sum, sizeof dst->tally, hipMemcpyDeviceToHost,
                          c->stream));
    return HTREE_OK;
}

htree_status htree::status_code(uint32_t word) {
    if (word & kStatusNonFinite) return fail(HTREE_EINVAL, "non-finite particle position");
    if (word & kStatusOverflow) return fail(HTREE_EOVERFLOW, "device capacity exceeded");
    return HTREE_OK;
}
