/*
 * htree_oracle.c -- FP64 CPU oracle for the force path of the hybrid
 * hard/soft tree method (Watanabe & Nakasato, "GPU accelerated Hybrid Tree
 * Algorithm for Collision-less N-body Simulations", arXiv:1406.6158).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain statement of what the GPU
 * library computes.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no source, header, table or helper with
 * the GPU library.
 *
 * Precision: IEEE binary64 round-to-nearest throughout, built with
 * -ffp-contract=off; every fused multiply-add that the tree contract
 * prescribes is written as fma().
 *
 * Layout: positions are structure-of-arrays, x[a*n + i] for axis a of
 * particle i.  Masses are float64.  Outputs are written in the caller's
 * particle order.
 *
 * Readings of the paper taken here (where it is silent or ambiguous):
 *  - the mass in the pair force is the source mass, and j = i is excluded;
 *  - the potential is the Plummer-softened -G m / sqrt(r^2 + eps^2);
 *  - the changeover K uses the unsoftened distance;
 *  - a cell is split iff it holds at least n_crit particles and is above
 *    level 21 (63-bit keys); the root is the power-of-two cube anchored at the
 *    coordinate minimum;
 *  - the opening radius is r_b = l / theta (cell side l) by default, or the
 *    paper's absolute MAC of section II.B (orc_tree_set_mac) with G kept in
 *    sqrt(3 G B2 / a_err); either way the paper's "open iff r_b > r" rule;
 *  - a sink group uses the distance from its bounding box, a lower bound of
 *    the paper's minimum over sinks, or (orc_tree_set_mac) that minimum;
 *  - in hybrid mode a cell is accepted only if every pair it stands for is
 *    at r >= R2; leaves nearer than that are summed particle by particle with
 *    the (1 - K) weight;
 *  - the two-timestep integrator is the nested kick-drift-kick.
 *
 * Parity status: every function below is pinned by a CPU test against closed
 * forms, invariants, brute force or library routines, except where its header
 * says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXLEVEL 21

int orc_version(void) { return 4; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Neumaier's compensated sum: s + c carries the running total. */
typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double nval(const nsum *a) { return a->s + a->c; }

/* ---------------------------------------------------------------------------
 * Changeover function, section II.C eq. (10):
 *   K = 1 for Y >= 1;  10 Y^6 - 15 Y^8 + 6 Y^10 for 0 < Y < 1;  0 for Y <= 0
 * with Y = (R2 - r) / (R2 - R1).
 * ------------------------------------------------------------------------- */
double orc_K(double Y)
{
    if (Y >= 1.0) return 1.0;
    if (Y <= 0.0) return 0.0;
    double Y2 = Y * Y;
    double Y6 = Y2 * Y2 * Y2;
    double Y8 = Y6 * Y2;
    double Y10 = Y8 * Y2;
    return 10.0 * Y6 - 15.0 * Y8 + 6.0 * Y10;
}

static inline double kY(double r, double R1, double R2)
{
    return orc_K((R2 - r) / (R2 - R1));
}

/* ---------------------------------------------------------------------------
 * Direct summation, section II.A eqs. (1)-(2): the acceleration of sink i is
 * the sum over sources j != i of G m_j (r_j - r_i) / (|r_i - r_j|^2 + eps^2)^{3/2}.
 * Optional potential sum of -G m_j / sqrt(r^2 + eps^2).
 *
 * sinks: ns caller indices (NULL means all n, ns must equal n); results are
 * written to acc[a*ns + k] and pot[k] for the k-th sink.
 * ------------------------------------------------------------------------- */
void orc_direct(int64_t n, const double *x, const double *m, double G, double eps,
                int64_t ns, const int64_t *sinks, double *acc, double *pot)
{
    const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ns; k++) {
        int64_t i = sinks ? sinks[k] : k;
        nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[j] - x[i];
            double dy = x[n + j] - x[n + i];
            double dz = x[2 * n + j] - x[2 * n + i];
            double r2 = dx * dx + dy * dy + dz * dz;
            double s2 = r2 + e2;
            double rinv = 1.0 / sqrt(s2);
            double f = G * m[j] * rinv * rinv * rinv;
            nadd(&ax, f * dx);
            nadd(&ay, f * dy);
            nadd(&az, f * dz);
            nadd(&ph, -G * m[j] * rinv);
        }
        acc[k] = nval(&ax);
        acc[ns + k] = nval(&ay);
        acc[2 * ns + k] = nval(&az);
        if (pot) pot[k] = nval(&ph);
    }
}

/* ---------------------------------------------------------------------------
 * Direct hard/soft split, section II.C eqs. (7)-(9):
 *   hard_i = sum over the neighbour set N(i) of K(r) F_ij
 *   soft_i = sum over all j != i of (1 - K(r)) F_ij
 * The neighbour set is N(i) = { j != i : r^2 < R2^2 } with
 *   r^2 = fma(dz, dz, fma(dy, dy, dx*dx)),  d = x_j - x_i  (FP64),
 * the exact test the GPU's neighbour search must reproduce bit for bit.
 * K vanishes at r >= R2, so hard_i is the full hard force.
 * Any of a_hard, a_soft, ngb may be NULL.
 * ------------------------------------------------------------------------- */
void orc_split_direct(int64_t n, const double *x, const double *m, double G, double eps,
                      double R1, double R2, int64_t ns, const int64_t *sinks,
                      double *a_hard, double *a_soft, int64_t *ngb)
{
    const double e2 = eps * eps;
    const double R2sq = R2 * R2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < ns; k++) {
        int64_t i = sinks ? sinks[k] : k;
        nsum hx = {0, 0}, hy = {0, 0}, hz = {0, 0};
        nsum sx = {0, 0}, sy = {0, 0}, sz = {0, 0};
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[j] - x[i];
            double dy = x[n + j] - x[n + i];
            double dz = x[2 * n + j] - x[2 * n + i];
            double r2c = fma(dz, dz, fma(dy, dy, dx * dx));
            int near = r2c < R2sq;
            if (!near && !a_soft) continue;
            double r2 = dx * dx + dy * dy + dz * dz;
            double rinv = 1.0 / sqrt(r2 + e2);
            double f = G * m[j] * rinv * rinv * rinv;
            double K = near ? kY(sqrt(r2), R1, R2) : 0.0;
            if (near) {
                cnt++;
                nadd(&hx, K * f * dx);
                nadd(&hy, K * f * dy);
                nadd(&hz, K * f * dz);
            }
            double w = (1.0 - K) * f;
            nadd(&sx, w * dx);
            nadd(&sy, w * dy);
            nadd(&sz, w * dz);
        }
        if (a_hard) {
            a_hard[k] = nval(&hx);
            a_hard[ns + k] = nval(&hy);
            a_hard[2 * ns + k] = nval(&hz);
        }
        if (a_soft) {
            a_soft[k] = nval(&sx);
            a_soft[ns + k] = nval(&sy);
            a_soft[2 * ns + k] = nval(&sz);
        }
        if (ngb) ngb[k] = cnt;
    }
}

/* ---------------------------------------------------------------------------
 * Energies: kinetic sum m v^2 / 2 and potential (1/2) sum_i m_i phi_i with the
 * direct softened potential (diagnostic of section IV.A's energy check).
 * ------------------------------------------------------------------------- */
void orc_energy(int64_t n, const double *x, const double *v, const double *m,
                double G, double eps, double *kin, double *pot)
{
    const double e2 = eps * eps;
    nsum ks = {0, 0}, ps = {0, 0};
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        nsum p = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[j] - x[i];
            double dy = x[n + j] - x[n + i];
            double dz = x[2 * n + j] - x[2 * n + i];
            double r2 = dx * dx + dy * dy + dz * dz;
            nadd(&p, -G * m[j] / sqrt(r2 + e2));
        }
        phi[i] = nval(&p);
    }
    for (int64_t i = 0; i < n; i++) {
        if (v) {
            double v2 = v[i] * v[i] + v[n + i] * v[n + i] + v[2 * n + i] * v[2 * n + i];
            nadd(&ks, 0.5 * m[i] * v2);
        }
        nadd(&ps, 0.5 * m[i] * phi[i]);
    }
    free(phi);
    if (kin) *kin = nval(&ks);
    if (pot) *pot = nval(&ps);
}

/* ===========================================================================
 * Tree (section II.B; construction as in section III.A.1)
 * ========================================================================= */

typedef struct {
    int32_t level;
    int32_t nchild;
    int64_t first, count;     /* particle range in sorted order            */
    int64_t parent;
    int64_t child[8];
    double M;                 /* cell mass                                 */
    double com[3];            /* centre of mass, build frame               */
    double blo[3];            /* cell box lower corner, build frame        */
    double l;                 /* cell side                                 */
    double rb2;               /* squared opening radius                    */
    double B2;                /* sum of m |COM - u|^2 over the cell (eq. 6) */
    double bmax2;             /* max |COM - u|^2 over the cell's particles  */
} onode;

typedef struct {
    int64_t n;
    int32_t n_crit;
    double theta, invth2;
    double lo[3], side;
    int64_t *perm;            /* sorted position -> caller index           */
    uint64_t *key;            /* Morton keys, sorted                       */
    uint32_t *q;              /* [3][n] quantised coordinates, sorted      */
    double *u;                /* [3][n] build-frame positions, sorted      */
    double *x;                /* [3][n] original positions, sorted         */
    double *m;                /* masses, sorted                            */
    onode *nd;
    int64_t nn, cap;
    int64_t *gstart;          /* sink groups: [gstart[k], gstart[k+1]) in sorted order */
    int64_t ng, gcap;
    int32_t g;
    int32_t mac_min;          /* group rule: 0 box distance, 1 minimum over sinks */
} orc_tree;

typedef struct { uint64_t key; int64_t idx; } kv;

static int kv_cmp(const void *a, const void *b)
{
    const kv *p = (const kv *)a, *q = (const kv *)b;
    if (p->key < q->key) return -1;
    if (p->key > q->key) return 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/* Interleave bits 20..0 of (qx, qy, qz): x takes the most significant slot. */
uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t k = 0;
    for (int b = ORC_MAXLEVEL - 1; b >= 0; b--) {
        k = (k << 3) | ((uint64_t)((qx >> b) & 1u) << 2)
                     | ((uint64_t)((qy >> b) & 1u) << 1)
                     | (uint64_t)((qz >> b) & 1u);
    }
    return k;
}

/* Smallest power of two >= ext (1 if ext == 0). */
static double pow2_ceil(double ext)
{
    if (!(ext > 0.0)) return 1.0;
    int e;
    double f = frexp(ext, &e);           /* ext = f 2^e, f in [0.5, 1) */
    return (f == 0.5) ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

/*
 * Build frame and keys (section III.A.1: root region, Morton keys, sort):
 *   lo_a = min x_a;  u = x - lo (one rounded subtraction per coordinate);
 *   side = smallest power of two >= max u;  q_a = min(floor(u_a 2^21 / side), 2^21 - 1);
 *   keys interleave q; stable sort by key.
 */
static void tree_keys(orc_tree *T, const double *x, const double *m)
{
    int64_t n = T->n;
    for (int a = 0; a < 3; a++) {
        double lo = n ? x[a * n] : 0.0;
        for (int64_t i = 1; i < n; i++) if (x[a * n + i] < lo) lo = x[a * n + i];
        T->lo[a] = lo;
    }
    double ext = 0.0;
    for (int a = 0; a < 3; a++)
        for (int64_t i = 0; i < n; i++) {
            double u = x[a * n + i] - T->lo[a];
            if (u > ext) ext = u;
        }
    T->side = pow2_ceil(ext);
    double scale = ldexp(1.0, ORC_MAXLEVEL) / T->side;   /* exact power of two */
    uint32_t qmax = (1u << ORC_MAXLEVEL) - 1u;
    uint32_t *qtmp = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)(n ? n : 1));
    kv *tab = (kv *)malloc(sizeof(kv) * (size_t)(n ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        uint32_t qq[3];
        for (int a = 0; a < 3; a++) {
            double u = x[a * n + i] - T->lo[a];
            double s = floor(u * scale);
            qq[a] = (s >= (double)qmax) ? qmax : (uint32_t)s;
            qtmp[a * n + i] = qq[a];
        }
        tab[i].key = orc_interleave(qq[0], qq[1], qq[2]);
        tab[i].idx = i;
    }
    qsort(tab, (size_t)n, sizeof(kv), kv_cmp);
    for (int64_t p = 0; p < n; p++) {
        int64_t i = tab[p].idx;
        T->perm[p] = i;
        T->key[p] = tab[p].key;
        T->m[p] = m[i];
        for (int a = 0; a < 3; a++) {
            T->q[a * n + p] = qtmp[a * n + i];
            T->x[a * n + p] = x[a * n + i];
            T->u[a * n + p] = x[a * n + i] - T->lo[a];
        }
    }
    free(qtmp);
    free(tab);
}

static int64_t new_node(orc_tree *T)
{
    if (T->nn == T->cap) {
        T->cap = T->cap ? 2 * T->cap : 1024;
        T->nd = (onode *)realloc(T->nd, sizeof(onode) * (size_t)T->cap);
    }
    memset(&T->nd[T->nn], 0, sizeof(onode));
    return T->nn++;
}

/*
 * Recursive 3-bit split (section III.A.1): a node holding the sorted range
 * [b, e) at level lev is a leaf if it has fewer than n_crit particles (or is at
 * the deepest level); otherwise its range is divided by the key digit of the
 * next level into up to eight non-empty children, taken in octant order.
 */
static int64_t split(orc_tree *T, int32_t lev, int64_t b, int64_t e, int64_t parent)
{
    int64_t id = new_node(T);
    T->nd[id].level = lev;
    T->nd[id].first = b;
    T->nd[id].count = e - b;
    T->nd[id].parent = parent;
    T->nd[id].nchild = 0;
    if (e - b < T->n_crit || lev == ORC_MAXLEVEL) return id;
    int shift = 3 * (ORC_MAXLEVEL - 1 - lev);
    int64_t s = b;
    for (uint64_t o = 0; o < 8; o++) {
        int64_t t = s;
        while (t < e && ((T->key[t] >> shift) & 7u) == o) t++;
        if (t > s) {
            int64_t c = split(T, lev + 1, s, t, id);
            int32_t k = T->nd[id].nchild++;
            T->nd[id].child[k] = c;
        }
        s = t;
    }
    return id;
}

/*
 * Cell moments (section II.B: centre of mass per cell) in the build frame,
 * summation order fixed:
 *   leaf:     M = sum m_i and S_a = fma(m_i, u_ia, S_a), in sorted order;
 *   internal: M and S summed over the children in octant order;
 *   COM = S / M (cell centre if M == 0).
 * Geometry: l = side 2^-level; box lower corner = (q >> (21 - level)) l;
 * squared opening radius r_b^2 = (l l) invtheta^2 with invtheta^2 = 1/theta^2.
 */
/* |p - q|^2 as fma(dz, dz, fma(dy, dy, dx * dx)), d = p - q. */
static inline double sqdist(const double *p, double qx, double qy, double qz)
{
    double dx = p[0] - qx, dy = p[1] - qy, dz = p[2] - qz;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

static void moments(orc_tree *T, int64_t id, double *Sout)
{
    onode *c = &T->nd[id];
    int64_t n = T->n;
    c->l = ldexp(T->side, -c->level);
    for (int a = 0; a < 3; a++)
        c->blo[a] = (double)(T->q[a * n + c->first] >> (ORC_MAXLEVEL - c->level)) * c->l;
    c->rb2 = (c->l * c->l) * T->invth2;
    double M = 0.0, S[3] = {0.0, 0.0, 0.0};
    if (c->nchild == 0) {
        for (int64_t i = c->first; i < c->first + c->count; i++) {
            M += T->m[i];
            for (int a = 0; a < 3; a++) S[a] = fma(T->m[i], T->u[a * n + i], S[a]);
        }
    } else {
        for (int k = 0; k < c->nchild; k++) {
            double Sc[3];
            moments(T, c->child[k], Sc);
            M += T->nd[c->child[k]].M;
            for (int a = 0; a < 3; a++) S[a] += Sc[a];
        }
    }
    c->M = M;
    for (int a = 0; a < 3; a++) {
        Sout[a] = S[a];
        c->com[a] = (M != 0.0) ? S[a] / M : c->blo[a] + 0.5 * c->l;
    }
    /* Quantities of the absolute MAC (section II.B, eqs. 5-6), in the build
     * frame.  B2 = sum_i m_i |COM - u_i|^2: a leaf sums its particles in
     * sorted order; an inner cell sums over its children in octant order
     * B2_c + M_c |COM - COM_c|^2 (the parallel-axis identity, equal to the
     * particle sum up to rounding).  bmax2 = max_i |COM - u_i|^2 over all the
     * cell's particles (a maximum: independent of order). */
    double B2 = 0.0, bm = 0.0;
    if (c->nchild == 0) {
        for (int64_t i = c->first; i < c->first + c->count; i++) {
            double q = sqdist(c->com, T->u[i], T->u[n + i], T->u[2 * n + i]);
            B2 = fma(T->m[i], q, B2);
        }
    } else {
        for (int k = 0; k < c->nchild; k++) {
            const onode *h = &T->nd[c->child[k]];
            double q = sqdist(c->com, h->com[0], h->com[1], h->com[2]);
            B2 = B2 + fma(h->M, q, h->B2);
        }
    }
    for (int64_t i = c->first; i < c->first + c->count; i++) {
        double q = sqdist(c->com, T->u[i], T->u[n + i], T->u[2 * n + i]);
        if (q > bm) bm = q;
    }
    c->B2 = B2;
    c->bmax2 = bm;
}

orc_tree *orc_tree_build(int64_t n, const double *x, const double *m, int32_t n_crit, double theta)
{
    if (n < 1 || n_crit < 1) return NULL;
    orc_tree *T = (orc_tree *)calloc(1, sizeof(orc_tree));
    T->n = n;
    T->n_crit = n_crit;
    T->theta = theta;
    T->invth2 = 1.0 / (theta * theta);
    size_t nn = (size_t)n;
    T->perm = (int64_t *)malloc(sizeof(int64_t) * nn);
    T->key = (uint64_t *)malloc(sizeof(uint64_t) * nn);
    T->q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * nn);
    T->u = (double *)malloc(sizeof(double) * 3 * nn);
    T->x = (double *)malloc(sizeof(double) * 3 * nn);
    T->m = (double *)malloc(sizeof(double) * nn);
    tree_keys(T, x, m);
    split(T, 0, 0, n, -1);
    double S[3];
    moments(T, 0, S);
    return T;
}

void orc_tree_free(orc_tree *T)
{
    if (!T) return;
    free(T->perm); free(T->key); free(T->q); free(T->u); free(T->x); free(T->m);
    free(T->nd);
    free(T->gstart);
    free(T);
}

int64_t orc_tree_nnodes(const orc_tree *T) { return T->nn; }

void orc_tree_frame(const orc_tree *T, double *lo3, double *side)
{
    for (int a = 0; a < 3; a++) lo3[a] = T->lo[a];
    *side = T->side;
}

void orc_tree_sorted(const orc_tree *T, int64_t *perm, uint64_t *key, double *u)
{
    int64_t n = T->n;
    if (perm) memcpy(perm, T->perm, sizeof(int64_t) * (size_t)n);
    if (key) memcpy(key, T->key, sizeof(uint64_t) * (size_t)n);
    if (u) memcpy(u, T->u, sizeof(double) * 3 * (size_t)n);
}

/* Node arrays in the oracle's own (depth-first) order; any pointer may be NULL. */
void orc_tree_nodes(const orc_tree *T, int32_t *level, int64_t *first, int64_t *count,
                    int64_t *parent, int32_t *nchild, double *M, double *com, double *blo,
                    double *l, double *rb2)
{
    int64_t nn = T->nn;
    for (int64_t k = 0; k < nn; k++) {
        const onode *c = &T->nd[k];
        if (level) level[k] = c->level;
        if (first) first[k] = c->first;
        if (count) count[k] = c->count;
        if (parent) parent[k] = c->parent;
        if (nchild) nchild[k] = c->nchild;
        if (M) M[k] = c->M;
        for (int a = 0; a < 3; a++) {
            if (com) com[a * nn + k] = c->com[a];
            if (blo) blo[a * nn + k] = c->blo[a];
        }
        if (l) l[k] = c->l;
        if (rb2) rb2[k] = c->rb2;
    }
}

/*
 * Opening radii and group rule (section II.B eq. 5, section III.A.2 eq. 11).
 * a_err > 0: the absolute MAC,
 *   r_b = b_max / 2 + sqrt(b_max^2 / 4 + sqrt(3 G B2 / a_err)),
 * evaluated as b = sqrt(bmax2), t = sqrt(((3 G) B2) / a_err),
 * r_b = 0.5 b + sqrt(0.25 bmax2 + t), rb2 = r_b * r_b (every sqrt correctly
 * rounded); a_err = 0: r_b = l / theta of the build.  min_sinks = 1: a group
 * measures a cell by the minimum over its sinks of |u_i - COM|^2 (the paper's
 * n_vec rule) instead of the distance from its bounding box.
 */
void orc_tree_set_mac(orc_tree *T, double a_err, double G, int32_t min_sinks)
{
    T->mac_min = min_sinks ? 1 : 0;
    for (int64_t k = 0; k < T->nn; k++) {
        onode *c = &T->nd[k];
        if (a_err > 0.0) {
            double b = sqrt(c->bmax2);
            double t = sqrt(((3.0 * G) * c->B2) / a_err);
            double rb = 0.5 * b + sqrt(0.25 * c->bmax2 + t);
            c->rb2 = rb * rb;
        } else {
            c->rb2 = (c->l * c->l) * T->invth2;
        }
    }
}

/* B2 and bmax2 of every node, in the order of orc_tree_nodes. */
void orc_tree_node_mac(const orc_tree *T, double *B2, double *bmax2)
{
    for (int64_t k = 0; k < T->nn; k++) {
        if (B2) B2[k] = T->nd[k].B2;
        if (bmax2) bmax2[k] = T->nd[k].bmax2;
    }
}

/* ===========================================================================
 * Sink groups (section III.A.2: several sinks share one traversal; their
 * positions must be close, which the key order provides)
 * ========================================================================= */

static void gpush(orc_tree *T, int64_t start)
{
    if (T->ng == T->gcap) {
        T->gcap = T->gcap ? 2 * T->gcap : 1024;
        T->gstart = (int64_t *)realloc(T->gstart, sizeof(int64_t) * (size_t)(T->gcap + 1));
    }
    T->gstart[T->ng++] = start;
}

/*
 * Groups of at most g sorted particles (reading of section III.A.2: the
 * sinks of a group are consecutive in key order and lie in one cell).  With
 * the chunking limit L = cells * g, the chunking cells are the cells with at
 * most L particles whose parent holds more (the root if it holds at most L),
 * and the leaves whose parent holds more: each is cut into consecutive
 * chunks of g particles, the last one shorter.  A cell of at most g particles
 * is therefore one group.
 */
static void groups_rec(orc_tree *T, int64_t id, int64_t g, int64_t lim)
{
    const onode *c = &T->nd[id];
    if (c->count <= lim || c->nchild == 0) {
        for (int64_t s = c->first; s < c->first + c->count; s += g) gpush(T, s);
        return;
    }
    for (int k = 0; k < c->nchild; k++) groups_rec(T, c->child[k], g, lim);
}

/* Builds the sink groups for group size g >= 1 and chunking limit
 * cells * g (cells >= 1); returns their number. */
int64_t orc_tree_groups(orc_tree *T, int32_t g, int32_t cells)
{
    T->ng = 0;
    T->g = g;
    groups_rec(T, 0, g, (int64_t)cells * g);
    T->gstart[T->ng] = T->n;
    return T->ng;
}

void orc_tree_group_starts(const orc_tree *T, int64_t *starts)
{
    memcpy(starts, T->gstart, sizeof(int64_t) * (size_t)(T->ng + 1));
}

/* ===========================================================================
 * Walk (section II.B traversal rule; section III.A.2 grouped sinks, eq. 11)
 * ========================================================================= */

typedef struct {
    double lo[3], hi[3];      /* sink-group bounding box, build frame */
    int64_t b, e;             /* the group's sinks (sorted positions)  */
} gbox;

static inline double gap_pt(double lo, double hi, double p)
{
    double g = fmax(lo - p, p - hi);
    return g > 0.0 ? g : 0.0;
}

static inline double gap_box(double glo, double ghi, double clo, double chi)
{
    double g = fmax(glo - chi, clo - ghi);
    return g > 0.0 ? g : 0.0;
}

static inline double d2(double gx, double gy, double gz)
{
    return fma(gz, gz, fma(gy, gy, gx * gx));
}

static void group_box(const orc_tree *T, int64_t b, int64_t e, gbox *B)
{
    int64_t n = T->n;
    B->b = b;
    B->e = e;
    for (int a = 0; a < 3; a++) {
        double lo = T->u[a * n + b], hi = lo;
        for (int64_t i = b + 1; i < e; i++) {
            double v = T->u[a * n + i];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        B->lo[a] = lo;
        B->hi[a] = hi;
    }
}

typedef struct {
    int64_t *pc, *far, *near;     /* node ids (p-c cells, far leaves, near leaves) */
    int64_t npc, nfar, nnear, cpc, cfar, cnear;
    int64_t pfar, pnear;          /* particle counts in far / near leaves */
} wlist;

static void push(int64_t **a, int64_t *n, int64_t *cap, int64_t v)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 256;
        *a = (int64_t *)realloc(*a, sizeof(int64_t) * (size_t)*cap);
    }
    (*a)[(*n)++] = v;
}

/*
 * Opening rule for a sink group and a cell c (the paper opens when r_b > r):
 *   D1 = dist^2(box_g, COM_c) (or, with min_sinks, min_i |u_i - COM_c|^2),
 *   D2 = dist^2(box_g, box_c)   (fma form above)
 *   accepted iff D1 >= r_b^2 and (hybrid ? D2 >= R2^2 : D2 > 0);
 * an accepted cell is one particle-cell term; a rejected leaf contributes its
 * particles ("near" iff hybrid and D2 < R2^2, else "far"); otherwise the
 * children are visited.
 */
static void walk(const orc_tree *T, int64_t id, const gbox *B, double R2sq, int hybrid, wlist *L)
{
    const onode *c = &T->nd[id];
    double D1;
    if (T->mac_min) {
        /* minimum over the group's sinks of |u_i - COM|^2 */
        int64_t n = T->n;
        D1 = INFINITY;
        for (int64_t i = B->b; i < B->e; i++) {
            double q = sqdist(c->com, T->u[i], T->u[n + i], T->u[2 * n + i]);
            if (q < D1) D1 = q;
        }
    } else {
        D1 = d2(gap_pt(B->lo[0], B->hi[0], c->com[0]),
                gap_pt(B->lo[1], B->hi[1], c->com[1]),
                gap_pt(B->lo[2], B->hi[2], c->com[2]));
    }
    double D2 = d2(gap_box(B->lo[0], B->hi[0], c->blo[0], c->blo[0] + c->l),
                   gap_box(B->lo[1], B->hi[1], c->blo[1], c->blo[1] + c->l),
                   gap_box(B->lo[2], B->hi[2], c->blo[2], c->blo[2] + c->l));
    int sep = hybrid ? (D2 >= R2sq) : (D2 > 0.0);
    if (D1 >= c->rb2 && sep) {
        push(&L->pc, &L->npc, &L->cpc, id);
        return;
    }
    if (c->nchild == 0) {
        if (hybrid && D2 < R2sq) {
            push(&L->near, &L->nnear, &L->cnear, id);
            L->pnear += c->count;
        } else {
            push(&L->far, &L->nfar, &L->cfar, id);
            L->pfar += c->count;
        }
        return;
    }
    for (int k = 0; k < c->nchild; k++) walk(T, c->child[k], B, R2sq, hybrid, L);
}

static void wl_free(wlist *L) { free(L->pc); free(L->far); free(L->near); }

/*
 * Per-group list sizes for the groups of orc_tree_groups: n_pc cells, n_far
 * and n_near source particles (self included).
 */
void orc_walk_counts(const orc_tree *T, double R2, int32_t hybrid,
                     int64_t *n_pc, int64_t *n_far, int64_t *n_near)
{
    int64_t ng = T->ng;
    double R2sq = R2 * R2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < ng; k++) {
        int64_t b = T->gstart[k], e = T->gstart[k + 1];
        gbox B;
        group_box(T, b, e, &B);
        wlist L;
        memset(&L, 0, sizeof(L));
        walk(T, 0, &B, R2sq, hybrid, &L);
        n_pc[k] = L.npc;
        n_far[k] = L.pfar;
        n_near[k] = L.pnear;
        wl_free(&L);
    }
}

/* Node-id lists of one group (for brute-force cross-checks); returns the three
 * counts in cnt[0..2] and writes up to cap ids into each non-NULL array. */
void orc_walk_group(const orc_tree *T, int64_t k, double R2, int32_t hybrid,
                    int64_t cap, int64_t *pc, int64_t *far, int64_t *near, int64_t *cnt)
{
    int64_t b = T->gstart[k], e = T->gstart[k + 1];
    gbox B;
    group_box(T, b, e, &B);
    wlist L;
    memset(&L, 0, sizeof(L));
    walk(T, 0, &B, R2 * R2, hybrid, &L);
    for (int64_t i = 0; i < L.npc && i < cap; i++) if (pc) pc[i] = L.pc[i];
    for (int64_t i = 0; i < L.nfar && i < cap; i++) if (far) far[i] = L.far[i];
    for (int64_t i = 0; i < L.nnear && i < cap; i++) if (near) near[i] = L.near[i];
    cnt[0] = L.npc;
    cnt[1] = L.nfar;
    cnt[2] = L.nnear;
    wl_free(&L);
}

/*
 * Soft force of the groups listed (all if groups == NULL; groups as built by
 * orc_tree_groups), section II.C with
 * the tree of section II.B:
 *   a_i = sum_cells G M_c (COM_c - u_i) / (d^2 + eps^2)^{3/2}
 *       + sum_far  j != i  G m_j (u_j - u_i) / (r^2 + eps^2)^{3/2}
 *       + sum_near j != i  (1 - K(r)) G m_j (u_j - u_i) / (r^2 + eps^2)^{3/2}
 * (plain mode: no near leaves, so this is the normal tree force).
 * pot_i is the unsplit potential over every list entry.
 * Results go to acc[a*n + caller index] and pot[caller index]; the
 * interaction count (sinks times entries, self pairs included) is returned.
 */
int64_t orc_soft(const orc_tree *T, double G, double eps, double R1, double R2,
                 int32_t hybrid, int64_t ngr, const int64_t *groups, double *acc, double *pot)
{
    int64_t n = T->n;
    if (!groups) ngr = T->ng;
    double e2 = eps * eps, R2sq = R2 * R2;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int64_t t = 0; t < ngr; t++) {
        int64_t k = groups ? groups[t] : t;
        int64_t b = T->gstart[k], e = T->gstart[k + 1];
        gbox B;
        group_box(T, b, e, &B);
        wlist L;
        memset(&L, 0, sizeof(L));
        walk(T, 0, &B, R2sq, hybrid, &L);
        total += (e - b) * (L.npc + L.pfar + L.pnear);
        for (int64_t i = b; i < e; i++) {
            nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0};
            double ux = T->u[i], uy = T->u[n + i], uz = T->u[2 * n + i];
            for (int64_t q = 0; q < L.npc; q++) {
                const onode *c = &T->nd[L.pc[q]];
                double dx = c->com[0] - ux, dy = c->com[1] - uy, dz = c->com[2] - uz;
                double r2 = dx * dx + dy * dy + dz * dz;
                double rinv = 1.0 / sqrt(r2 + e2);
                double f = G * c->M * rinv * rinv * rinv;
                nadd(&ax, f * dx); nadd(&ay, f * dy); nadd(&az, f * dz);
                nadd(&ph, -G * c->M * rinv);
            }
            for (int pass = 0; pass < 2; pass++) {
                int64_t cnt = pass ? L.nnear : L.nfar;
                const int64_t *lv = pass ? L.near : L.far;
                for (int64_t q = 0; q < cnt; q++) {
                    const onode *c = &T->nd[lv[q]];
                    for (int64_t j = c->first; j < c->first + c->count; j++) {
                        if (j == i) continue;
                        double dx = T->u[j] - ux, dy = T->u[n + j] - uy, dz = T->u[2 * n + j] - uz;
                        double r2 = dx * dx + dy * dy + dz * dz;
                        double rinv = 1.0 / sqrt(r2 + e2);
                        double f = G * T->m[j] * rinv * rinv * rinv;
                        double w = pass ? (1.0 - kY(sqrt(r2), R1, R2)) * f : f;
                        nadd(&ax, w * dx); nadd(&ay, w * dy); nadd(&az, w * dz);
                        nadd(&ph, -G * T->m[j] * rinv);
                    }
                }
            }
            int64_t ci = T->perm[i];
            acc[ci] = nval(&ax);
            acc[n + ci] = nval(&ay);
            acc[2 * n + ci] = nval(&az);
            if (pot) pot[ci] = nval(&ph);
        }
        wl_free(&L);
    }
    return total;
}

/* ===========================================================================
 * Integrator (section II.A eqs. 3-4; two timesteps, section II.C)
 * ========================================================================= */

/* Full force used by the integrator: soft tree force plus the direct hard
 * force (hybrid), or the plain tree force. Writes a_s and a_h (caller order). */
static void forces(int64_t n, const double *x, const double *m, double G, double eps,
                   double theta, double R1, double R2, int32_t n_crit, int32_t g, int32_t cells,
                   int32_t hybrid, double *a_s, double *a_h)
{
    orc_tree *T = orc_tree_build(n, x, m, n_crit, theta);
    orc_tree_groups(T, g, cells);
    orc_soft(T, G, eps, R1, R2, hybrid, 0, NULL, a_s, NULL);
    orc_tree_free(T);
    if (hybrid)
        orc_split_direct(n, x, m, G, eps, R1, R2, n, NULL, a_h, NULL, NULL);
    else
        memset(a_h, 0, sizeof(double) * 3 * (size_t)n);
}

/*
 * Nested kick-drift-kick over n_soft soft steps of dt_soft, each split into
 * n_sub hard substeps of dt_h = dt_soft / n_sub (one soft-step plus
 * n_sub - 1 hard-steps per dt_soft):
 *   v += dt_s/2 a_s
 *   repeat n_sub times:
 *       v += dt_h/2 a_h;  x += dt_h v;
 *       last substep: a_s = soft(x), a_h = hard(x); otherwise a_h = hard(x)
 *       v += dt_h/2 a_h
 *   v += dt_s/2 a_s
 * Plain mode (hybrid = 0) is the same loop with a_s the full tree force and
 * a_h = 0.  Forces at the initial positions are computed first.  x, v are
 * updated in place (caller order).
 */
void orc_step(int64_t n, double *x, double *v, const double *m, double G, double eps,
              double theta, double R1, double R2, int32_t n_crit, int32_t g, int32_t cells,
              int32_t hybrid,
              double dt_soft, int32_t n_sub, int32_t n_soft)
{
    size_t s3 = sizeof(double) * 3 * (size_t)n;
    double *a_s = (double *)malloc(s3), *a_h = (double *)malloc(s3);
    double dt_h = dt_soft / n_sub;
    forces(n, x, m, G, eps, theta, R1, R2, n_crit, g, cells, hybrid, a_s, a_h);
    for (int32_t s = 0; s < n_soft; s++) {
        for (int64_t k = 0; k < 3 * n; k++) v[k] += 0.5 * dt_soft * a_s[k];
        for (int32_t h = 0; h < n_sub; h++) {
            for (int64_t k = 0; k < 3 * n; k++) v[k] += 0.5 * dt_h * a_h[k];
            for (int64_t k = 0; k < 3 * n; k++) x[k] += dt_h * v[k];
            if (h == n_sub - 1) {
                forces(n, x, m, G, eps, theta, R1, R2, n_crit, g, cells, hybrid, a_s, a_h);
            } else if (hybrid) {
                orc_split_direct(n, x, m, G, eps, R1, R2, n, NULL, a_h, NULL, NULL);
            }
            for (int64_t k = 0; k < 3 * n; k++) v[k] += 0.5 * dt_h * a_h[k];
        }
        for (int64_t k = 0; k < 3 * n; k++) v[k] += 0.5 * dt_soft * a_s[k];
    }
    free(a_s);
    free(a_h);
}
