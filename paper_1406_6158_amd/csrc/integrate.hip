// integrate.hip -- leapfrog kick/drift (section II.A eqs. 3-4) and the
// caller-order <-> key-order layout kernels.  All are HBM-streaming kernels:
// one thread per particle, coalesced structure-of-arrays accesses.
#include "htree_dev.h"

namespace htree {

constexpr int kNT = 256;

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kNT - 1) / kNT)); }

// v += c1 a1 + c2 a2 (FP32; either term may be absent), then x += dt v (FP64).
// v += c1 a1 + c2 a2 (FP32), then x += dt v (FP64); the packed copy xm of
// the positions (with the masses m) follows the drift.
__global__ __launch_bounds__(kNT) void k_kick_drift(double *x, double4 *xm, const float *m,
                                                    float *v, const float *a1, float c1,
                                                    const float *a2, float c2, double dt,
                                                    int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    double xn[3];
    for (int a = 0; a < 3; a++) {
        float vv = v[a * n + i];
        if (a1) vv = vv + c1 * a1[a * n + i];
        if (a2) vv = vv + c2 * a2[a * n + i];
        v[a * n + i] = vv;
        if (dt != 0.0) {
            xn[a] = x[a * n + i] + dt * (double)vv;
            x[a * n + i] = xn[a];
        }
    }
    if (dt != 0.0 && xm) xm[i] = make_double4(xn[0], xn[1], xn[2], (double)m[i]);
}

void launch_kick_drift(double *x, double4 *xm, const float *m, float *v, const float *a1, float c1,
                       const float *a2, float c2, double dt_drift, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_kick_drift, grid_for(n), dim3(kNT), 0, s, x, xm, m, v, a1, c1, a2, c2,
                       dt_drift, n);
}

__global__ __launch_bounds__(kNT) void k_scatter3(const float *src, const uint32_t *perm,
                                                  float *dst, int64_t n) {
    int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= n) return;
    uint32_t c = perm[p];
    dst[c] = src[p];
    dst[n + c] = src[n + p];
    dst[2 * n + c] = src[2 * n + p];
}

void launch_scatter3(const float *src_sorted, const uint32_t *perm, float *dst, int64_t n,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_scatter3, grid_for(n), dim3(kNT), 0, s, src_sorted, perm, dst, n);
}

template <typename T>
__global__ __launch_bounds__(kNT) void k_scatter1(const T *src, const uint32_t *perm, T *dst,
                                                  int64_t n) {
    int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= n) return;
    dst[perm[p]] = src[p];
}

void launch_scatter1f(const float *src_sorted, const uint32_t *perm, float *dst, int64_t n,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_scatter1<float>, grid_for(n), dim3(kNT), 0, s, src_sorted, perm, dst, n);
}

void launch_scatter1i(const int32_t *src_sorted, const uint32_t *perm, int32_t *dst, int64_t n,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_scatter1<int32_t>, grid_for(n), dim3(kNT), 0, s, src_sorted, perm, dst,
                       n);
}

__global__ __launch_bounds__(kNT) void k_gather3(const float *src, const uint32_t *perm,
                                                 float *dst, int64_t n) {
    int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= n) return;
    uint32_t c = perm[p];
    dst[p] = src[c];
    dst[n + p] = src[n + c];
    dst[2 * n + p] = src[2 * n + c];
}

void launch_gather3(const float *src_caller, const uint32_t *perm, float *dst_sorted, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_gather3, grid_for(n), dim3(kNT), 0, s, src_caller, perm, dst_sorted, n);
}

__global__ __launch_bounds__(kNT) void k_scatter_x(const double *xs, const uint32_t *perm,
                                                   double *dst, int64_t n) {
    int64_t p = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (p >= n) return;
    uint32_t c = perm[p];
    dst[c] = xs[p];
    dst[n + c] = xs[n + p];
    dst[2 * n + c] = xs[2 * n + p];
}

void launch_scatter_x(const double *x_sorted, const uint32_t *perm, double *dst, int64_t n,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_x, grid_for(n), dim3(kNT), 0, s, x_sorted, perm, dst, n);
}

__global__ __launch_bounds__(kNT) void k_set_state(const double *x, int64_t ldx, const float *v,
                                                   const float *m, double *xs, float *vs,
                                                   float *ms, uint32_t *perm, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 3; a++) {
        xs[a * n + i] = x[a * ldx + i];
        vs[a * n + i] = v ? v[a * n + i] : 0.0f;
    }
    ms[i] = m[i];
    perm[i] = (uint32_t)i;
}

void launch_set_state(const double *x, int64_t ldx, const float *v, const float *m, double *xs,
                      float *vs, float *ms, uint32_t *perm, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_state, grid_for(n), dim3(kNT), 0, s, x, ldx, v, m, xs, vs, ms, perm,
                       n);
}

__global__ __launch_bounds__(kNT) void k_add3(const float *a, const float *b, float *out,
                                              int64_t n3) {
    int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= n3) return;
    out[i] = a[i] + b[i];
}

void launch_add3(const float *a, const float *b, float *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_add3, grid_for(3 * n), dim3(kNT), 0, s, a, b, out, 3 * n);
}

__global__ __launch_bounds__(kNT) void k_zero_u32(uint32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < n) p[i] = 0u;
}

void launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, grid_for(n), dim3(kNT), 0, s, p, n);
}

}  // namespace htree
