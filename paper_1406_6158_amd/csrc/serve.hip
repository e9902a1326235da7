// serve.hip -- request server: continuous batching of independent force
// solves on one GPU.
//
// A request is one full force solve (build + soft force, + hard force in
// hybrid mode) of its own particle system.  Requests queue in arrival order;
// the head of the queue is admitted as soon as a device slot is free and the
// arena has a contiguous block for its footprint (context workspace plus
// outputs).  Admitted requests run on the caller's streams, up to per_stream
// of them queued on each, so one request's tree build overlaps another's walk
// and interactions on the device.  Completion is detected with one event per
// slot; finished results stay in the arena until the caller releases them.
//
// Single-threaded: all calls on one server come from one host thread with
// the server's device current.
#include <hip/hip_runtime.h>

#include "../../include/htree.h"
#include "arena.h"
#include "internal.h"

#include <stdarg.h>
#include <stdio.h>

#include <chrono>
#include <deque>
#include <unordered_map>
#include <vector>

using namespace htree;

namespace {

constexpr int32_t kMaxStreams = 64;
constexpr int32_t kMaxPerStream = 16;

htree_status err(htree_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
htree_status err(htree_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

#define SRV_HIP(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return err(HTREE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Byte layout of one admitted request inside its arena block.
struct Layout {
    size_t ws, acc_soft, acc_hard, ngb, pot, total;
};

Layout layout_of(const htree_params *p, int64_t n) {
    Layout L{};
    size_t off = 0;
    auto put = [&](size_t bytes) {
        size_t at = off;
        off += Arena::round_up(bytes);
        return at;
    };
    size_t ws = htree_workspace_bytes(p, n);
    if (ws == 0) return L;
    L.ws = put(ws);
    L.acc_soft = put(12 * (size_t)n);
    if (p->hybrid) {
        L.acc_hard = put(12 * (size_t)n);
        L.ngb = put(4 * (size_t)n);
    } else {
        L.acc_hard = L.ngb = Arena::kNone;
    }
    L.pot = (p->flags & HTREE_F_POT) ? put(4 * (size_t)n) : Arena::kNone;
    L.total = off;
    return L;
}

enum class St { pending, running, done, failed };

struct Request {
    htree_params p;
    int64_t n;
    const double *x;
    int64_t ldx;
    const float *m;
    hipEvent_t ready = nullptr;    // recorded on the inputs' stream at submission
    St state = St::pending;
    htree_status status = HTREE_OK;
    Layout L{};
    size_t off = Arena::kNone;
    htree_ctx *ctx = nullptr;
    int32_t slot = -1, stream = -1;
    double t_submit = 0, t_admit = 0, t_done = 0;
    unsigned long long tally[4] = {0, 0, 0, 0};
};

}  // namespace

struct htree_server {
    char *base = nullptr;
    Arena arena{0};
    std::vector<hipStream_t> streams;
    std::vector<int32_t> load;            // requests running per stream
    int32_t per_stream = 1;
    std::vector<hipEvent_t> slot_ev;      // one completion event per slot
    std::vector<hipEvent_t> ev_free;      // input-ready events not in use
    std::vector<int64_t> slot_req;        // request running in each slot, -1 if free
    CtxReport *report = nullptr;          // pinned, one per slot
    std::deque<int64_t> queue;            // pending, arrival order
    std::unordered_map<int64_t, Request> req;
    std::deque<int64_t> finished;         // completed, not yet reported by poll
    int64_t next_id = 1;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    htree_server_stats st{};
};

namespace {

double now_s(const htree_server *s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

// Returns a request's input-ready event to the pool (its wait, if any, was
// enqueued before the request's own completion, so it has long been met).
void drop_ready(htree_server *s, Request &r) {
    if (r.ready) s->ev_free.push_back(r.ready);
    r.ready = nullptr;
}

void finish(htree_server *s, int64_t id, Request &r, htree_status code) {
    drop_ready(s, r);
    r.status = code;
    r.state = code == HTREE_OK ? St::done : St::failed;
    r.t_done = now_s(s);
    if (code != HTREE_OK) {
        // a failed solve keeps nothing: its context and block go back now
        if (r.ctx) htree_destroy(r.ctx);
        r.ctx = nullptr;
        if (r.off != Arena::kNone) s->arena.release(r.off);
        r.off = Arena::kNone;
        s->st.failed++;
    } else {
        s->st.completed++;
    }
    s->finished.push_back(id);
}

htree_status enqueue_solve(htree_server *s, Request &r, char *blk, hipStream_t strm);

// Enqueues the whole solve of r on its stream; the slot event marks the end.
htree_status launch(htree_server *s, Request &r) {
    char *blk = s->base + r.off;
    hipStream_t strm = s->streams[r.stream];
    // the solve reads the inputs only after the work that wrote them
    SRV_HIP(hipStreamWaitEvent(strm, r.ready, 0));
    htree_status e = htree_create(&r.ctx, &r.p, r.n, blk + r.L.ws, htree_workspace_bytes(&r.p, r.n),
                                  strm);
    if (e) return e;
    e = enqueue_solve(s, r, blk, strm);
    if (e) {
        // work may already be queued on the stream: let it end before the
        // block can be handed to another request
        (void)hipStreamSynchronize(strm);
    }
    return e;
}

htree_status enqueue_solve(htree_server *s, Request &r, char *blk, hipStream_t strm) {
    htree_status e;
    if ((e = ctx_set_state(r.ctx, r.x, r.ldx, nullptr, r.m))) return e;
    if ((e = htree_build_tree(r.ctx))) return e;
    float *pot = r.L.pot != Arena::kNone ? (float *)(blk + r.L.pot) : nullptr;
    if ((e = htree_soft_force(r.ctx, (float *)(blk + r.L.acc_soft), pot))) return e;
    if (r.p.hybrid &&
        (e = htree_hard_force(r.ctx, (float *)(blk + r.L.acc_hard), (int32_t *)(blk + r.L.ngb))))
        return e;
    if ((e = ctx_report_async(r.ctx, &s->report[r.slot]))) return e;
    SRV_HIP(hipEventRecord(s->slot_ev[r.slot], strm));
    return HTREE_OK;
}

// Moves finished slots to the finished list, then admits from the queue head.
htree_status pump(htree_server *s) {
    for (size_t k = 0; k < s->slot_req.size(); k++) {
        int64_t id = s->slot_req[k];
        if (id < 0) continue;
        hipError_t q = hipEventQuery(s->slot_ev[k]);
        if (q == hipErrorNotReady) continue;
        Request &r = s->req[id];
        s->slot_req[k] = -1;
        s->load[r.stream]--;
        s->st.in_flight--;
        if (q != hipSuccess) {
            finish(s, id, r, err(HTREE_EDEVICE, "request %lld: %s", (long long)id,
                                 hipGetErrorString(q)));
            continue;
        }
        const CtxReport &rep = s->report[k];
        for (int j = 0; j < 4; j++) r.tally[j] = rep.tally[j];
        finish(s, id, r, status_code(rep.status));
    }
    while (!s->queue.empty()) {
        // a free slot on the least loaded stream
        int32_t best = -1;
        for (int32_t k = 0; k < (int32_t)s->streams.size(); k++)
            if (s->load[k] < s->per_stream && (best < 0 || s->load[k] < s->load[best])) best = k;
        if (best < 0) break;
        int64_t id = s->queue.front();
        Request &r = s->req[id];
        size_t off = s->arena.alloc(r.L.total);
        if (off == Arena::kNone) break;    // strict arrival order: wait for memory
        s->queue.pop_front();
        s->st.pending--;
        r.off = off;
        r.stream = best;
        r.slot = -1;
        for (int32_t k = 0; k < (int32_t)s->slot_req.size(); k++)
            if (s->slot_req[k] < 0) {
                r.slot = k;
                break;
            }
        r.state = St::running;
        r.t_admit = now_s(s);
        s->st.admitted++;
        htree_status e = launch(s, r);
        if (e) {
            // nothing was recorded on the slot event; the request ends here
            finish(s, id, r, e);
            continue;
        }
        s->slot_req[r.slot] = id;
        s->load[best]++;
        s->st.in_flight++;
        if (s->st.in_flight > s->st.peak_in_flight) s->st.peak_in_flight = s->st.in_flight;
    }
    s->st.bytes_in_use = s->arena.used();
    s->st.bytes_peak = s->arena.peak();
    return HTREE_OK;
}

}  // namespace

extern "C" {

size_t htree_solve_footprint(const htree_params *p, int64_t n) {
    if (!p) return 0;
    return layout_of(p, n).total;
}

htree_status htree_server_create(htree_server **out, void *d_arena, size_t arena_bytes,
                                 void *const *hip_streams, int32_t n_streams,
                                 int32_t per_stream) {
    if (!out) return err(HTREE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_arena || ((uintptr_t)d_arena & 255u))
        return err(HTREE_EINVAL, "arena must be non-NULL and 256-byte aligned");
    if (!hip_streams || n_streams < 1 || n_streams > kMaxStreams)
        return err(HTREE_EINVAL, "n_streams must be in [1, %d]", kMaxStreams);
    if (per_stream < 1 || per_stream > kMaxPerStream)
        return err(HTREE_EINVAL, "per_stream must be in [1, %d]", kMaxPerStream);
    htree_server *s = new htree_server();
    s->base = (char *)d_arena;
    s->arena = Arena(arena_bytes);
    s->per_stream = per_stream;
    for (int32_t k = 0; k < n_streams; k++) s->streams.push_back((hipStream_t)hip_streams[k]);
    s->load.assign(n_streams, 0);
    const int32_t slots = n_streams * per_stream;
    s->slot_req.assign(slots, -1);
    s->t0 = std::chrono::steady_clock::now();
    s->st.arena_bytes = s->arena.size();
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->report, sizeof(CtxReport) * slots);
    for (int32_t k = 0; k < slots && e == hipSuccess; k++) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) s->slot_ev.push_back(ev);
    }
    if (e != hipSuccess) {
        htree_server_destroy(s);
        return err(HTREE_EDEVICE, "server setup: %s", hipGetErrorString(e));
    }
    *out = s;
    return HTREE_OK;
}

htree_status htree_server_submit(htree_server *s, const htree_params *p, int64_t n,
                                 const double *d_x, int64_t ldx, const float *d_m,
                                 void *hip_input_stream, int64_t *id) {
    if (!s || !p || !id) return err(HTREE_EINVAL, "server, params or id is NULL");
    *id = 0;
    if (!d_x || !d_m) return err(HTREE_EINVAL, "x and m are required");
    if (ldx < n) return err(HTREE_EINVAL, "x row stride %lld < n", (long long)ldx);
    if (p->flags & HTREE_F_TIMING) return err(HTREE_EINVAL, "HTREE_F_TIMING is not served");
    Layout L = layout_of(p, n);
    if (L.total == 0) {
        // report the parameter error itself
        htree_workspace_bytes(p, n);
        return HTREE_EINVAL;
    }
    if (L.total > s->arena.size())
        return err(HTREE_ENOMEM, "footprint %zu bytes exceeds the arena (%zu)", L.total,
                   s->arena.size());
    Request r;
    if (s->ev_free.empty()) {
        hipEvent_t ev;
        SRV_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        s->ev_free.push_back(ev);
    }
    r.ready = s->ev_free.back();
    SRV_HIP(hipEventRecord(r.ready, (hipStream_t)hip_input_stream));
    s->ev_free.pop_back();
    r.p = *p;
    r.n = n;
    r.x = d_x;
    r.ldx = ldx;
    r.m = d_m;
    r.L = L;
    r.t_submit = now_s(s);
    *id = s->next_id++;
    s->req.emplace(*id, r);
    s->queue.push_back(*id);
    s->st.submitted++;
    s->st.pending++;
    return pump(s);
}

htree_status htree_server_poll(htree_server *s, int64_t *done, int32_t max_done,
                               int32_t *n_done) {
    if (!s || !n_done || (max_done > 0 && !done)) return err(HTREE_EINVAL, "bad arguments");
    *n_done = 0;
    htree_status e = pump(s);
    while (*n_done < max_done && !s->finished.empty()) {
        done[(*n_done)++] = s->finished.front();
        s->finished.pop_front();
    }
    return e;
}

htree_status htree_server_result(htree_server *s, int64_t id, htree_request_info *info,
                                 float **d_acc_soft, float **d_acc_hard, int32_t **d_ngb,
                                 float **d_pot) {
    if (!s) return err(HTREE_EINVAL, "server is NULL");
    auto it = s->req.find(id);
    if (it == s->req.end()) return err(HTREE_EINVAL, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (info) {
        info->n = r.n;
        info->status = r.status;
        info->state = (int32_t)r.state;
        info->stream = r.stream;
        info->t_submit = r.t_submit;
        info->t_admit = r.t_admit;
        info->t_done = r.t_done;
        info->footprint = r.L.total;
        info->soft_interactions = (int64_t)r.tally[0];
        info->hard_candidates = (int64_t)r.tally[1];
        info->hard_pairs = (int64_t)r.tally[2];
    }
    char *blk = r.state == St::done ? s->base + r.off : nullptr;
    auto at = [&](size_t o) { return blk && o != Arena::kNone ? blk + o : nullptr; };
    if (d_acc_soft) *d_acc_soft = (float *)at(r.L.acc_soft);
    if (d_acc_hard) *d_acc_hard = (float *)at(r.L.acc_hard);
    if (d_ngb) *d_ngb = (int32_t *)at(r.L.ngb);
    if (d_pot) *d_pot = (float *)at(r.L.pot);
    if (r.state == St::pending || r.state == St::running)
        return err(HTREE_ESTATE, "request %lld has not finished", (long long)id);
    return r.status;
}

htree_status htree_server_release(htree_server *s, int64_t id) {
    if (!s) return err(HTREE_EINVAL, "server is NULL");
    auto it = s->req.find(id);
    if (it == s->req.end()) return err(HTREE_EINVAL, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (r.state == St::running)
        return err(HTREE_ESTATE, "request %lld is running", (long long)id);
    if (r.state == St::pending) {
        for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
            if (*q == id) {
                s->queue.erase(q);
                break;
            }
        s->st.pending--;
        s->st.cancelled++;
        drop_ready(s, r);
    } else {
        for (auto q = s->finished.begin(); q != s->finished.end(); ++q)
            if (*q == id) {
                s->finished.erase(q);
                break;
            }
        if (r.ctx) htree_destroy(r.ctx);
        if (r.off != Arena::kNone) s->arena.release(r.off);
    }
    s->req.erase(it);
    return pump(s);
}

htree_status htree_server_get_stats(htree_server *s, htree_server_stats *out) {
    if (!s || !out) return err(HTREE_EINVAL, "server or out is NULL");
    s->st.held = 0;
    for (auto &kv : s->req)
        if (kv.second.state == St::done) s->st.held++;
    s->st.bytes_in_use = s->arena.used();
    s->st.bytes_peak = s->arena.peak();
    *out = s->st;
    return HTREE_OK;
}

void htree_server_destroy(htree_server *s) {
    if (!s) return;
    for (size_t k = 0; k < s->slot_req.size(); k++)
        if (s->slot_req[k] >= 0) (void)hipEventSynchronize(s->slot_ev[k]);
    for (auto &kv : s->req) {
        if (kv.second.ctx) htree_destroy(kv.second.ctx);
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    }
    for (hipEvent_t e : s->slot_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_free) (void)hipEventDestroy(e);
    if (s->report) (void)hipHostFree(s->report);
    delete s;
}

}  // extern "C"
