/*
 * htree.h -- C ABI of the MI355X (gfx950) library for the force path of the
 * hybrid hard/soft tree method (Watanabe & Nakasato, arXiv:1406.6158).
 *
 * The method (section II):
 *   - softened gravity, eq. (2): the acceleration of sink i from source j is
 *     G m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}, j != i;
 *   - the force is split by the changeover K(r) of eq. (10) into a hard part
 *     F K (neighbours inside R2) and a soft part F (1 - K), eqs. (7)-(9);
 *   - the soft part comes from a Barnes-Hut octree walk (section II.B, with
 *     grouped sinks as in section III.A.2), the hard part from a neighbour
 *     search within R2 and a direct K-weighted sum;
 *   - a leapfrog (section II.A eqs. 3-4) applies the hard force every
 *     substep dt_h and the soft force every dt_s = n dt_h (section II.C).
 *
 * Conventions shared by every entry point:
 *   - All pointers named d_* are DEVICE pointers on the device that is
 *     current when htree_create is called.  Positions are float64,
 *     velocities, masses and accelerations float32, all structure-of-arrays:
 *     component a of particle i is at [a*n + i].  Arrays the caller passes are
 *     in the caller's particle order; the library keeps its own
 *     Morton-sorted copy and translates.
 *   - The caller owns every device buffer, including the one workspace the
 *     library carves its internal arrays from.  The library never allocates or
 *     frees device memory; it owns only the small host-side context.
 *   - Every call that launches work is asynchronous on the HIP stream given
 *     to htree_create and returns once the work is enqueued.  Host-detectable
 *     errors are returned at once; conditions found on the device are kept in
 *     a sticky status word that htree_sync returns.
 *   - A context is not thread-safe.  Separate contexts on separate streams
 *     may be used concurrently.
 *   - On error, htree_last_error() returns a text for the calling thread.
 */
#ifndef HTREE_H
#define HTREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t htree_status;
#define HTREE_OK         0
#define HTREE_EINVAL    (-1)  /* bad parameter or shape, or non-finite input      */
#define HTREE_ENOMEM    (-2)  /* workspace smaller than htree_workspace_bytes     */
#define HTREE_EDEVICE   (-3)  /* HIP runtime error (text in htree_last_error)     */
#define HTREE_EOVERFLOW (-4)  /* a device-side capacity was exceeded              */
#define HTREE_ESTATE    (-5)  /* call order: e.g. soft_force before build_tree    */

/* htree_params.flags */
#define HTREE_F_POT     1     /* soft_force also evaluates the tree potential     */
#define HTREE_F_TIMING  2     /* record per-phase times with HIP events           */
#define HTREE_F_REUSE   4     /* hard force: reuse the search between builds      */
                              /* (htree_hard_force describes it)                  */

typedef struct {
    double  G;            /* gravitational constant (> 0)                            */
    double  eps;          /* Plummer softening length (>= 1e-15)                     */
    double  theta;        /* opening angle: a cell of side l is opened while the     */
                          /* group lies closer than l/theta; 0 opens every cell     */
    double  R1, R2;       /* changeover band, 0 < R1 < R2 (hybrid mode only)         */
    double  dt_soft;      /* soft timestep dt_s                                      */
    int32_t n_sub;        /* hard substeps per soft step, dt_h = dt_s / n_sub (>= 1) */
    int32_t hybrid;       /* 1: hard/soft split; 0: plain tree (normal-tree mode)    */
    int32_t n_crit;       /* a cell splits while it holds >= n_crit particles (>= 1) */
    int32_t group_size;   /* at most this many sinks share one walk, 1..64 (64: one  */
                          /* sink per lane of a wavefront)                          */
    int32_t precision;    /* soft interactions: 0 FP32 with compensated tile sums;   */
                          /* 1 FP64 (results are still stored as FP32); the hard    */
                          /* force always sums its pair terms in FP64               */
    int32_t flags;        /* HTREE_F_*                                               */
    int32_t group_cell;   /* soft sink groups: the chunking cells are the cells of   */
                          /* at most group_cell * group_size particles whose parent */
                          /* holds more, and the leaves whose parent holds more;    */
                          /* each is cut into chunks of group_size (1..4096)        */
    int32_t group_mac;    /* how a sink group measures a cell for the opening test:  */
                          /* 0 the distance from the group's bounding box to the    */
                          /* centre of mass; 1 the minimum over the group's sinks   */
                          /* of their distance to it (section III.A.2, eq. 11)      */
    double  a_err;        /* 0: opening radius l / theta; > 0: the absolute MAC of   */
                          /* section II.B (eqs. 5-6), r_b = b_max/2 + sqrt(b_max^2/4 */
                          /* + sqrt(3 G B2 / a_err)), theta then unused             */
} htree_params;

typedef struct {
    int64_t n, n_groups, n_nodes, n_leaves;
    int64_t soft_cells;         /* particle-cell entries, summed over groups        */
    int64_t soft_far;           /* far particle entries, summed over groups         */
    int64_t soft_near;          /* near (1-K weighted) particle entries             */
    int64_t soft_interactions;  /* sum over groups of sinks x entries               */
    int64_t hard_candidates;    /* sink-source pairs tested against R2              */
    int64_t hard_pairs;         /* accepted neighbour pairs (sum of ngb)            */
    float   ms_build, ms_soft, ms_hard, ms_kick;  /* summed, with HTREE_F_TIMING  */
    int32_t calls_build, calls_soft, calls_hard, pad;
} htree_counters;

typedef struct htree_ctx htree_ctx;

/* Defaults: G = 1, eps = 0.01, theta = 0.5, R1 = 0.05, R2 = 0.1, dt_soft = 1/16,
 * n_sub = 4, hybrid = 1, n_crit = 16, group_size = 64, precision = 0, flags = 0,
 * group_cell = 16, group_mac = 0, a_err = 0. */
void htree_default_params(htree_params *p);

/* Exact number of workspace bytes a context for n particles needs (0 if the
 * parameters are invalid).  This is the device footprint used for admission. */
size_t htree_workspace_bytes(const htree_params *p, int64_t n);

/* Batch of S independent systems in one context (one launch per phase serves
 * all of them).  p[s] and n[s] describe system s (1 <= S <= 65536, total
 * particles <= 2^27).  G, eps, theta, R1, R2, n_crit and group_size may
 * differ between systems; dt_soft, n_sub, hybrid, precision and flags must
 * equal those of system 0.  Particle arrays passed to the other calls concatenate
 * the systems in order: system s occupies positions [n_0 + ... + n_{s-1},
 * ... + n_s) of every [3][N] or [N] array (N = total).  Systems never
 * interact.  Same errors as htree_create; 0 bytes if invalid. */
size_t htree_batch_workspace_bytes(const htree_params *p, const int64_t *n, int32_t S);
htree_status htree_batch_create(htree_ctx **ctx, const htree_params *p, const int64_t *n,
                                int32_t S, void *d_workspace, size_t ws_bytes, void *hip_stream);
int32_t htree_system_count(htree_ctx *ctx);

/* Creates a context for n >= 1 particles.  d_workspace must hold ws_bytes >=
 * htree_workspace_bytes(p, n) bytes, 256-byte aligned, and stay valid until
 * htree_destroy.  hip_stream is a hipStream_t (NULL: the null stream).
 * Errors: EINVAL (params), ENOMEM (workspace too small), EDEVICE. */
htree_status htree_create(htree_ctx **ctx, const htree_params *p, int64_t n,
                          void *d_workspace, size_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * htree_create for one system of n particles, but the workspace is the
 * library's own static device array of 64 MiB (HTREE_STATIC_SCRATCH_BYTES),
 * one per device, held from its first use until the process ends.  No device
 * memory is allocated by this call or by any later call on the context; the
 * caller still passes every input and output buffer.  The limit: n must need
 * at most that many workspace bytes (htree_workspace_bytes; about 920 bytes
 * per particle with n_crit = 16, so n <= 2^16 fits), else ENOMEM.  One context
 * per device may hold the array at a time: ESTATE while another is alive.
 * htree_destroy of such a context first waits for its stream, so the next
 * one does not overwrite work still running.  The array keeps the last
 * context's contents; everything a context needs zeroed is cleared on the
 * device at creation.  Contexts on different devices are independent.
 * Errors: EINVAL, ENOMEM, ESTATE, EDEVICE. */
#define HTREE_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
htree_status htree_create_static(htree_ctx **ctx, const htree_params *p, int64_t n,
                                 void *hip_stream);

/* Copies the particle state in.  d_x [3][n] float64, d_v [3][n] float32 (may be
 * NULL: zero velocities), d_m [n] float32.  Invalidates the tree and forces. */
htree_status htree_set_state(htree_ctx *ctx, const double *d_x, const float *d_v,
                             const float *d_m);

/* Builds the octree of the current positions (section III.A.1): bounding box,
 * 63-bit Morton keys in the power-of-two root cube, stable radix sort,
 * recursive split while a cell holds >= n_crit particles, centres of mass in
 * FP64 and opening radii.  Reorders the internal state into key order. */
htree_status htree_build_tree(htree_ctx *ctx);

/* Soft force (hybrid) or full tree force (plain) at the positions of the last
 * build (section II.B traversal, section II.C split).  The result is kept
 * for the integrator and, if d_acc is not NULL, written in caller order
 * ([3][n] float32).  d_pot (float32 [n], may be NULL) receives the tree
 * potential when the context has HTREE_F_POT.  ESTATE without a current tree. */
htree_status htree_soft_force(htree_ctx *ctx, float *d_acc, float *d_pot);

/* Hard force, section II.C: for every sink the exact neighbour set
 * { j != i : |x_j - x_i|^2 < R2^2 } (FP64 test) and the sum of K(r) F_ij.
 * With HTREE_F_REUSE, the first launch after a build records each group's
 * search (the tree nodes it tests and does not open, with the opening radius
 * widened by R2/4) and the launches after htree_refit replay it against the
 * refitted boxes instead of walking from the root; the neighbour sets stay
 * exact, the pair terms are summed in another order.
 * Kept for the integrator; written in caller order if d_acc / d_ngb (int32
 * neighbour counts) are not NULL.  ESTATE without a current tree; EINVAL in
 * plain mode. */
htree_status htree_hard_force(htree_ctx *ctx, float *d_acc, int32_t *d_ngb);

/* Leapfrog update, section II.A eqs. (3)-(4): v += dt_kick * a, then
 * x += dt_drift * v (FP64 positions).  d_acc is [3][n] float32 in caller
 * order; NULL means the sum of the kept soft and hard accelerations.  A
 * non-zero dt_drift invalidates the tree. */
htree_status htree_kick_drift(htree_ctx *ctx, double dt_kick, const float *d_acc,
                              double dt_drift);

/* Advances n_soft_steps soft steps with the nested kick-drift-kick of
 * section II.C (one soft-step plus n_sub - 1 hard-steps per dt_s): per soft
 * step v += dt_s/2 a_s; n_sub times { v += dt_h/2 a_h; x += dt_h v;
 * last substep: rebuild, a_s = soft, a_h = hard; other substeps: refit the
 * node boxes to the drifted positions (same tree and groups), a_h = hard;
 * v += dt_h/2 a_h }; v += dt_s/2 a_s.  The hard force's neighbour sets are
 * exact either way.  Plain mode: n_sub = 1 with the full tree force.  Forces
 * at the initial positions are computed on the first call.  Kicks that meet
 * between two substeps (the closing half-kicks of one and the opening ones of
 * the next, with the same forces) are applied as one update, so the
 * velocities differ from separate half-kicks by FP32 rounding only. */
htree_status htree_step(htree_ctx *ctx, int32_t n_soft_steps);

/* Recomputes the node boxes of the last build at the current positions:
 * the same tree, particle order and groups, with boxes that bound the drifted
 * particles.  This is what the hard substeps of section II.C need (the hard
 * force is evaluated after every drift of dt_h, the tree is rebuilt only for
 * the soft force): after htree_kick_drift, htree_refit makes
 * htree_hard_force valid again (its neighbour sets stay exact); the soft
 * force still needs htree_build_tree.  ESTATE if no tree was built since
 * htree_set_state. */
htree_status htree_refit(htree_ctx *ctx);

/* Copies positions / velocities out in caller order (either may be NULL). */
htree_status htree_get_state(htree_ctx *ctx, double *d_x, float *d_v);

/* Waits for the context's stream and returns the sticky device status
 * (HTREE_OK, or EINVAL for non-finite input, EOVERFLOW). */
htree_status htree_sync(htree_ctx *ctx);

/* Counters summed over the build / force calls since the previous
 * htree_stats call (or since htree_create), after which they restart from
 * zero; n_nodes is that of the last build.  With HTREE_F_TIMING the ms_*
 * fields are the summed HIP-event times of each phase on the context's
 * stream.  Synchronises the stream. */
htree_status htree_stats(htree_ctx *ctx, htree_counters *out);

/* Opening-test quantities of the last build's nodes, in the order of
 * htree_export_nodes (host arrays, any may be NULL): B2 = sum m |COM - u|^2
 * (a leaf over its particles in sorted order, an inner node as the sum over
 * its children of B2_c + M_c |COM - COM_c|^2), bmax2 = the largest
 * |COM - u|^2 over the node's particles, and the squared opening radius rb2.
 * B2 and bmax2 are computed only when some system has a_err > 0 (else 0).
 * Synchronises the stream. */
htree_status htree_export_node_mac(htree_ctx *ctx, double *B2, double *bmax2, double *rb2);

/* Soft sink groups of the last build (section III.A.2: sinks that share one
 * traversal; these are the groups of the soft force and of its list sizes).
 * With g = group_size and L = group_cell * g: the chunking cells are the
 * cells of at most L particles whose parent holds more (the root if it holds
 * at most L) and the leaves whose parent holds more; each chunking cell is
 * cut into consecutive chunks of g particles in sorted order (the last one
 * shorter), and every chunk is a group.  htree_group_count returns their
 * number (-1 on error); htree_export_groups writes the count + 1 start
 * positions (sorted order, the last one n) to a host array.  Both
 * synchronise the stream.  (The hard force groups its sinks by a rule of its
 * own, which does not change any result.) */
int64_t htree_group_count(htree_ctx *ctx);
htree_status htree_export_groups(htree_ctx *ctx, int32_t *starts);

/* Per-group list sizes of the last soft_force: cells, far and near particle
 * entries (host arrays of htree_group_count int32 each; any may be NULL).
 * Synchronises the stream. */
htree_status htree_group_counts(htree_ctx *ctx, int32_t *n_cells, int32_t *n_far,
                                int32_t *n_near);

/* Copies the sorted keys, the permutation (sorted position -> caller index)
 * and the build frame of every system (lo[3], side: 4 doubles per system) of
 * the last build to host memory (any pointer may be NULL).  Synchronises the
 * stream. */
htree_status htree_export_keys(htree_ctx *ctx, uint64_t *keys, int32_t *perm,
                               double *frame4);

/* Number of tree nodes of the last build, and their records in level order
 * (host arrays of that length; any pointer may be NULL): level, first
 * particle (sorted position), particle count, mass, centre of mass [3][nn]
 * (build frame).  Synchronises the stream. */
int64_t htree_node_count(htree_ctx *ctx);
htree_status htree_export_nodes(htree_ctx *ctx, int32_t *level, int32_t *first,
                                int32_t *count, double *mass, double *com);

/* Bounding boxes of the nodes' particles at the positions they were last
 * computed for (the build, or htree_refit after a drift), in the order of
 * htree_export_nodes: lo and hi are host arrays [3][nn] (either may be NULL)
 * of the exact per-axis minima and maxima of the particles' FP64 positions.
 * These are the boxes the hard search of section II.C tests against R2.
 * ESTATE if they do not fit the current positions (a drift without a refit
 * or a build).  Synchronises the stream. */
htree_status htree_export_node_boxes(htree_ctx *ctx, double *lo, double *hi);

const char *htree_last_error(void);

/* Releases the host context; the caller then frees the workspace. */
void htree_destroy(htree_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of independent force solves.
 *
 * Not a construct of the paper: it serves many solves of the paper's force
 * (build, soft force and, in hybrid mode, hard force, as htree_build_tree /
 * htree_soft_force / htree_hard_force define them) of different sizes on one
 * GPU.  Requests queue in submission order.  The head of the queue is admitted
 * when a device slot is free (n_streams x per_stream slots) and the arena has
 * a contiguous block of htree_solve_footprint bytes; admission is strictly in
 * order.  An admitted request is enqueued whole on the least loaded stream, so
 * requests on different streams overlap on the device.  Its results stay in
 * its arena block until htree_server_release.  A request's results do not
 * depend on what else is in flight.
 *
 * One host thread per server, with the server's device current.  The library
 * allocates no device memory: the arena and the streams are the caller's and
 * must outlive the server.  The only allocation is a small pinned host buffer
 * (one 64-byte report per slot).
 * ------------------------------------------------------------------------- */
typedef struct htree_server htree_server;

typedef struct {
    int64_t submitted, admitted, completed, failed, cancelled;
    int64_t pending;          /* queued, not yet admitted                        */
    int64_t in_flight;        /* admitted, running on the device                 */
    int64_t held;             /* finished, results not yet released              */
    int64_t peak_in_flight;
    uint64_t arena_bytes, bytes_in_use, bytes_peak;
} htree_server_stats;

typedef struct {
    int64_t n;
    int32_t status;           /* HTREE_OK or the solve's error                   */
    int32_t state;            /* 0 pending, 1 running, 2 done, 3 failed          */
    int32_t stream;           /* index of the stream it ran on, -1 if none       */
    int32_t pad;
    double t_submit, t_admit, t_done;   /* host clock, seconds since server
                                           creation; t_done is when a poll saw
                                           the solve finished                    */
    uint64_t footprint;       /* arena bytes held                                */
    int64_t soft_interactions, hard_candidates, hard_pairs;
} htree_request_info;

/* Arena bytes one solve of n particles with params p holds while admitted:
 * its context workspace, acc_soft [3][n] f32, in hybrid mode acc_hard [3][n]
 * f32 and ngb [n] i32, with HTREE_F_POT pot [n] f32, each 256-byte aligned.
 * 0 if p or n is invalid. */
size_t htree_solve_footprint(const htree_params *p, int64_t n);

/* Creates a server over the device range d_arena[0, arena_bytes) (256-byte
 * aligned) and n_streams (1..64) caller streams (hipStream_t), with at most
 * per_stream (1..16) requests queued on each.  EINVAL, EDEVICE. */
htree_status htree_server_create(htree_server **srv, void *d_arena, size_t arena_bytes,
                                 void *const *hip_streams, int32_t n_streams,
                                 int32_t per_stream);

/* Queues one solve: d_x holds the x, y and z rows of the positions, ldx >= n
 * doubles apart (the first n of each row are used); d_m [n] f32 masses.  Both
 * must stay valid until the request has finished.  hip_input_stream is the
 * stream (hipStream_t, NULL: the null stream) on which the work that writes
 * d_x and d_m was enqueued: the solve reads them only after everything
 * enqueued on that stream before this call (an event recorded there now, and
 * waited for on the solve's stream).  HTREE_F_TIMING is rejected.  Writes the
 * request id (> 0).  EINVAL for bad parameters, ENOMEM if the footprint
 * exceeds the whole arena (never admissible), EDEVICE.  Admits what it can
 * before returning. */
htree_status htree_server_submit(htree_server *srv, const htree_params *p, int64_t n,
                                 const double *d_x, int64_t ldx, const float *d_m,
                                 void *hip_input_stream, int64_t *id);

/* Non-blocking: detects finished solves, admits queued ones, and writes up to
 * max_done ids of requests that finished (or failed) since they were last
 * reported into done[], their number into *n_done. */
htree_status htree_server_poll(htree_server *srv, int64_t *done, int32_t max_done,
                               int32_t *n_done);

/* Information and device result pointers of a request (any output pointer
 * may be NULL).  The arrays are in the caller's particle order and stay valid
 * until htree_server_release; pointers that do not apply (hard results of a
 * plain solve, pot without HTREE_F_POT, any result of an unfinished or failed
 * request) are set to NULL.  Returns the solve's status, ESTATE while it has
 * not finished, EINVAL for an unknown id. */
htree_status htree_server_result(htree_server *srv, int64_t id, htree_request_info *info,
                                 float **d_acc_soft, float **d_acc_hard, int32_t **d_ngb,
                                 float **d_pot);

/* Releases a finished request's arena block, or cancels a queued one.
 * ESTATE while it runs; EINVAL for an unknown id. */
htree_status htree_server_release(htree_server *srv, int64_t id);

htree_status htree_server_get_stats(htree_server *srv, htree_server_stats *out);

/* Waits for running solves, then frees the server (not the arena). */
void htree_server_destroy(htree_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HTREE_H */
