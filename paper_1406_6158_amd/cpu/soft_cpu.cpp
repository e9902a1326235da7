// soft_cpu.cpp -- the soft interaction loops on host CPU threads, for the
// CPU/GPU comparison of section IV.C (the paper runs its force kernels on both
// kinds of device).  This is a separate host library used by the benchmark
// and its tests; the HIP library never calls it and it is never a substitute
// for the GPU path.
//
// The arithmetic is that of the GPU soft kernel's interaction loops: sources
// are offsets from the group centre with their mass, in FP32; a far source (a
// cell monopole or a particle of a far leaf) adds
//     m (q - u) / (|q - u|^2 + eps^2)^{3/2}
// to sink u (section II.C eq. 9 with the unit weight); a near source (a
// particle of a leaf within R2 of the group box) adds the same times
// 1 - K(|q - u|) (eqs. 7-8), with K from the quintic S(Y^2), Y = (R2 - r) /
// (R2 - R1) clamped to [0, 1], and 1 - S(s) = S(1 - s).  Each tile of 64
// sources is summed plainly and added to the running sums with compensated
// (Kahan) summation.  The weight is evaluated only for a source that some of
// the 8 sinks of a vector have within R2 (beyond it the weight is exactly 1).
//
// Layout: 8 sinks per AVX2 vector (the GPU's lane = sink), two vectors at a
// time over the source list; groups are split over host threads.
#include <immintrin.h>

#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

namespace {

constexpr int kSinks = 64;   // sinks per group
constexpr int kTile = 64;    // sources per compensated partial sum

struct Sum8 {
    __m256 s[3], c[3];
};

inline void kahan8(__m256 &s, __m256 &c, __m256 v) {
    const __m256 y = _mm256_sub_ps(v, c);
    const __m256 t = _mm256_add_ps(s, y);
    c = _mm256_sub_ps(_mm256_sub_ps(t, s), y);
    s = t;
}

// 1 / sqrt(x) to FP32 accuracy: the hardware estimate and one Newton step.
inline __m256 rsqrt8(__m256 x) {
    const __m256 y = _mm256_rsqrt_ps(x);
    const __m256 h = _mm256_mul_ps(_mm256_set1_ps(0.5f), x);
    const __m256 yy = _mm256_mul_ps(y, y);
    return _mm256_mul_ps(y, _mm256_fnmadd_ps(h, yy, _mm256_set1_ps(1.5f)));
}

// 1 - K(r) as the GPU kernel forms it: w = 1 - Y^2, (10 - 15 w + 6 w^2) w^3.
inline __m256 one_minus_K8(__m256 r, __m256 R2, __m256 invdR) {
    __m256 Y = _mm256_mul_ps(_mm256_sub_ps(R2, r), invdR);
    Y = _mm256_min_ps(_mm256_max_ps(Y, _mm256_setzero_ps()), _mm256_set1_ps(1.0f));
    const __m256 w = _mm256_fnmadd_ps(Y, Y, _mm256_set1_ps(1.0f));
    const __m256 t = _mm256_fmadd_ps(_mm256_fmadd_ps(_mm256_set1_ps(6.0f), w, _mm256_set1_ps(-15.0f)),
                                     w, _mm256_set1_ps(10.0f));
    return _mm256_mul_ps(t, _mm256_mul_ps(w, _mm256_mul_ps(w, w)));
}

struct Consts {
    __m256 eps2, R2, invdR, u2skip;
};

// Two sink vectors (16 sinks: ux[2], uy[2], uz[2]) against cnt sources.
template <bool NEAR>
void tile2(const float *src, int64_t cnt, const __m256 *ux, const __m256 *uy, const __m256 *uz,
           const Consts &K, Sum8 *acc) {
    for (int64_t t0 = 0; t0 < cnt; t0 += kTile) {
        const int64_t t1 = t0 + kTile < cnt ? t0 + kTile : cnt;
        __m256 a[2][3];
        for (int v = 0; v < 2; v++)
            for (int k = 0; k < 3; k++) a[v][k] = _mm256_setzero_ps();
        for (int64_t j = t0; j < t1; j++) {
            const __m256 qx = _mm256_set1_ps(src[4 * j]), qy = _mm256_set1_ps(src[4 * j + 1]),
                         qz = _mm256_set1_ps(src[4 * j + 2]), qm = _mm256_set1_ps(src[4 * j + 3]);
            for (int v = 0; v < 2; v++) {
                const __m256 dx = _mm256_sub_ps(qx, ux[v]), dy = _mm256_sub_ps(qy, uy[v]),
                             dz = _mm256_sub_ps(qz, uz[v]);
                __m256 f;
                if (!NEAR) {
                    const __m256 r2 = _mm256_fmadd_ps(
                        dz, dz, _mm256_fmadd_ps(dy, dy, _mm256_fmadd_ps(dx, dx, K.eps2)));
                    const __m256 ri = rsqrt8(r2);
                    f = _mm256_mul_ps(_mm256_mul_ps(qm, ri), _mm256_mul_ps(ri, ri));
                } else {
                    const __m256 u2 =
                        _mm256_fmadd_ps(dz, dz, _mm256_fmadd_ps(dy, dy, _mm256_mul_ps(dx, dx)));
                    const __m256 ri = rsqrt8(_mm256_add_ps(u2, K.eps2));
                    f = _mm256_mul_ps(_mm256_mul_ps(qm, ri), _mm256_mul_ps(ri, ri));
                    if (_mm256_movemask_ps(_mm256_cmp_ps(u2, K.u2skip, _CMP_LT_OQ)))
                        f = _mm256_mul_ps(f, one_minus_K8(_mm256_sqrt_ps(u2), K.R2, K.invdR));
                }
                a[v][0] = _mm256_fmadd_ps(f, dx, a[v][0]);
                a[v][1] = _mm256_fmadd_ps(f, dy, a[v][1]);
                a[v][2] = _mm256_fmadd_ps(f, dz, a[v][2]);
            }
        }
        for (int v = 0; v < 2; v++)
            for (int k = 0; k < 3; k++) kahan8(acc[v].s[k], acc[v].c[k], a[v][k]);
    }
}

void group(const float *sinks, const float *far, int64_t nf, const float *near, int64_t nn,
           const Consts &K, float *out) {
    for (int b = 0; b < kSinks; b += 16) {
        __m256 ux[2], uy[2], uz[2];
        for (int v = 0; v < 2; v++) {
            ux[v] = _mm256_loadu_ps(sinks + b + 8 * v);
            uy[v] = _mm256_loadu_ps(sinks + kSinks + b + 8 * v);
            uz[v] = _mm256_loadu_ps(sinks + 2 * kSinks + b + 8 * v);
        }
        Sum8 acc[2];
        for (int v = 0; v < 2; v++)
            for (int k = 0; k < 3; k++) acc[v].s[k] = acc[v].c[k] = _mm256_setzero_ps();
        if (nf > 0) tile2<false>(far, nf, ux, uy, uz, K, acc);
        if (nn > 0) tile2<true>(near, nn, ux, uy, uz, K, acc);
        for (int v = 0; v < 2; v++)
            for (int k = 0; k < 3; k++)
                _mm256_storeu_ps(out + k * kSinks + b + 8 * v,
                                 _mm256_sub_ps(acc[v].s[k], acc[v].c[k]));
    }
}

}  // namespace

extern "C" {

// Soft accelerations (without the factor G) of ng groups of 64 sinks.
//   sinks [ng][3][64]  sink offsets from their group's centre (x row, y row, z row)
//   far   [ng][nf][4]  far sources of each group: x, y, z offsets and mass
//   near  [ng][nn][4]  near sources (weighted by 1 - K); nf or nn may be 0
//   eps2 = eps^2, R2, invdR = 1 / (R2 - R1); out [ng][3][64]
// Host pointers, owned by the caller.  Groups are split over `threads` host
// threads (at least 1).  Returns 0, or -1 for a negative size or a null
// pointer where data is needed.
int htree_cpu_soft(int32_t ng, const float *sinks, const float *far, int64_t nf,
                   const float *near, int64_t nn, float eps2, float R2, float invdR, float *out,
                   int32_t threads) {
    if (ng < 0 || nf < 0 || nn < 0) return -1;
    if (ng > 0 && (!sinks || !out || (nf > 0 && !far) || (nn > 0 && !near))) return -1;
    if (threads < 1) threads = 1;
    Consts K;
    K.eps2 = _mm256_set1_ps(eps2);
    K.R2 = _mm256_set1_ps(R2);
    K.invdR = _mm256_set1_ps(invdR);
    K.u2skip = _mm256_set1_ps(R2 * R2 * (1.0f + 0x1p-18f));
    auto work = [&](int32_t g0, int32_t g1) {
        for (int32_t g = g0; g < g1; g++)
            group(sinks + (int64_t)g * 3 * kSinks, far ? far + (int64_t)g * nf * 4 : nullptr, nf,
                  near ? near + (int64_t)g * nn * 4 : nullptr, nn, K,
                  out + (int64_t)g * 3 * kSinks);
    };
    if (threads == 1 || ng < 2) {
        work(0, ng);
        return 0;
    }
    std::vector<std::thread> pool;
    const int32_t per = (ng + threads - 1) / threads;
    for (int32_t t = 0; t < threads; t++) {
        const int32_t g0 = t * per, g1 = g0 + per < ng ? g0 + per : ng;
        if (g0 >= g1) break;
        pool.emplace_back(work, g0, g1);
    }
    for (auto &th : pool) th.join();
    return 0;
}

}  // extern "C"
