// Host emulation of the subset of the HIP device model and runtime that
// libhtree uses, for CPU tests of the unchanged kernel sources (built with
// g++ -std=c++20 and HTREE_EMU_CHECKS, which turns the kernels' HT_CHECK
// invariants into aborts).  TEST INFRASTRUCTURE ONLY: it is found instead of
// the real <hip/hip_runtime.h> through an -I path of the emulation build and
// is never part of the GPU library.
//
// Model:
//   - "device" memory is host memory; copies are memcpy; streams and events
//     are synchronous (events keep a host timestamp);
//   - a launch runs its blocks one after another; the threads of a block are
//     fibers (user-level contexts on the calling OS thread, switched by a few
//     instructions of x86-64 assembly) run by a round-robin scheduler;
//   - __syncthreads is a barrier over the live threads of the block, and every
//     cross-lane operation (ballot, shuffles, readlane, readfirstlane, DPP row
//     moves) is an exchange through a per-wavefront buffer between two
//     barriers over the live lanes of that wavefront; a barrier opens when
//     every live participant has arrived;
//   - a thread that returns from the kernel leaves the barriers, like a lane
//     whose execution ended; if no thread can run and no barrier can open
//     (threads of one block or wavefront waiting at different barriers), the
//     emulation reports a deadlock and aborts;
//   - __shared__ variables are function statics: blocks never run
//     concurrently;
//   - the hardware reciprocal square root and square root are the correctly
//     rounded host ones (the GPU's are approximations), so results agree with
//     the GPU to rounding, not bit for bit.
#pragma once

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <tuple>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __launch_bounds__(...)
#define __forceinline__ inline
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct alignas(16) float4 { float x, y, z, w; };
struct alignas(16) double4 { double x, y, z, w; };
struct alignas(8) uint2 { unsigned x, y; };
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }
inline double4 make_double4(double a, double b, double c, double d) { return {a, b, c, d}; }
inline uint2 make_uint2(unsigned a, unsigned b) { return {a, b}; }

// Context switch (x86-64 System V): saves the callee-saved registers and the
// stack pointer of the running context in *from, resumes the context whose
// stack pointer is `to`.  A new context starts in emu_fiber_start with its
// Fiber pointer in r12.  Weak symbols: every translation unit that includes
// this header emits them, the linker keeps one.
extern "C" void emu_switch(void **from, void *to);
extern "C" void emu_fiber_start();
asm(R"(
    .text
    .weak emu_switch
    .type emu_switch, @function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_switch, .-emu_switch
    .weak emu_fiber_start
    .type emu_fiber_start, @function
emu_fiber_start:
    movq %r12, %rdi
    andq $-16, %rsp
    call emu_fiber_main
    ud2
    .size emu_fiber_start, .-emu_fiber_start
)");

namespace emu {

constexpr int kWave = 64;
constexpr size_t kStack = 256 * 1024;

enum class FS { ready, wait_block, wait_wave, done };

struct Fiber {
    void *sp = nullptr;
    std::vector<char> stack;
    FS st = FS::done;
    int tid = 0;
};

struct Block {
    int nthreads = 0, nwaves = 0;
    std::vector<uint64_t> slot;       // kWave per wavefront
};

inline dim3 g_grid, g_dim, g_block_idx;
inline Block *g_blk = nullptr;
inline std::vector<Fiber> g_fib;      // one per thread of the running block
inline int g_cur = -1;                // running fiber, -1: the scheduler
inline void *g_sched_sp = nullptr;
inline const std::function<void(int)> *g_job = nullptr;

inline Fiber &cur() { return g_fib[g_cur]; }

// Back to the scheduler with the running fiber in state s.
inline void yield(FS s) {
    Fiber &f = cur();
    f.st = s;
    emu_switch(&f.sp, g_sched_sp);
}

inline void prepare(Fiber &f, int tid) {
    if (f.stack.empty()) f.stack.resize(kStack);
    uintptr_t top = ((uintptr_t)f.stack.data() + f.stack.size()) & ~(uintptr_t)15;
    void **sp = (void **)(top - 64);
    // popped by emu_switch: r15, r14, r13, r12 (= the fiber), rbx, rbp; then
    // the return address
    sp[0] = sp[1] = sp[2] = nullptr;
    sp[3] = &f;
    sp[4] = sp[5] = nullptr;
    sp[6] = (void *)&emu_fiber_start;
    f.sp = sp;
    f.st = FS::ready;
    f.tid = tid;
}

// Runs the threads of one block until all have returned.
inline void run_block(int n) {
    if ((int)g_fib.size() < n) g_fib.resize(n);
    for (int k = 0; k < n; k++) prepare(g_fib[k], k);
    const int nw = (n + kWave - 1) / kWave;
    for (;;) {
        bool ran = false;
        for (int k = 0; k < n; k++) {
            if (g_fib[k].st != FS::ready) continue;
            g_cur = k;
            emu_switch(&g_sched_sp, g_fib[k].sp);
            g_cur = -1;
            ran = true;
        }
        // open the barriers every live participant has reached
        bool any_live = false, opened = false;
        bool all_block = true;
        for (int k = 0; k < n; k++) {
            if (g_fib[k].st == FS::done) continue;
            any_live = true;
            if (g_fib[k].st != FS::wait_block) all_block = false;
        }
        if (!any_live) return;
        if (all_block) {   // (no live lane can wait at a wavefront barrier then)
            for (int k = 0; k < n; k++)
                if (g_fib[k].st == FS::wait_block) g_fib[k].st = FS::ready;
            opened = true;
        }
        for (int w = 0; w < nw; w++) {
            bool live = false, all = true;
            for (int k = w * kWave; k < n && k < (w + 1) * kWave; k++) {
                if (g_fib[k].st == FS::done) continue;
                live = true;
                if (g_fib[k].st != FS::wait_wave) all = false;
            }
            if (live && all) {
                for (int k = w * kWave; k < n && k < (w + 1) * kWave; k++)
                    if (g_fib[k].st == FS::wait_wave) g_fib[k].st = FS::ready;
                opened = true;
            }
        }
        if (!opened && !ran) {
            fprintf(stderr, "emu: deadlock in block %u: threads wait at different barriers\n",
                    g_block_idx.x);
            abort();
        }
    }
}

template <typename... KA, typename... A>
void launch(void (*k)(KA...), dim3 grid, dim3 block, A &&...args) {
    if (grid.y != 1 || grid.z != 1 || block.y != 1 || block.z != 1) {
        fprintf(stderr, "emu: only 1-D launches\n");
        abort();
    }
    if (grid.x == 0) return;
    g_grid = grid;
    g_dim = block;
    const int n = (int)block.x;
    const int nw = (n + kWave - 1) / kWave;
    std::tuple<KA...> targs(std::forward<A>(args)...);   // converted once, like kernel arguments
    std::function<void(int)> job = [&](int) { std::apply(k, targs); };
    g_job = &job;
    for (unsigned b = 0; b < grid.x; b++) {
        Block B;
        B.nthreads = n;
        B.nwaves = nw;
        B.slot.assign((size_t)nw * kWave, 0);
        g_blk = &B;
        g_block_idx = dim3(b);
        run_block(n);
        g_blk = nullptr;
    }
    g_job = nullptr;
}

inline dim3 thread_idx() { return dim3((unsigned)cur().tid); }
inline int lane() { return cur().tid % kWave; }
inline int wave() { return cur().tid / kWave; }

inline void block_barrier() { yield(FS::wait_block); }
inline void wave_barrier() { yield(FS::wait_wave); }

// Every lane of the wavefront publishes v; f reads the published values.
template <typename F>
inline uint64_t exchange(uint64_t v, F f) {
    uint64_t *s = g_blk->slot.data() + (size_t)wave() * kWave;
    s[lane()] = v;
    wave_barrier();
    const uint64_t r = f(s);
    wave_barrier();
    return r;
}

template <typename T>
inline uint64_t bits(T v) {
    static_assert(sizeof(T) <= 8, "exchange width");
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    return u;
}
template <typename T>
inline T from_bits(uint64_t u) {
    T v;
    memcpy(&v, &u, sizeof(T));
    return v;
}
inline int width() {
    const int rest = g_blk->nthreads - wave() * kWave;
    return rest < kWave ? rest : kWave;
}

inline uint64_t ballot(bool p) {
    const int w = width();
    return exchange(p ? 1u : 0u, [w](const uint64_t *s) {
        uint64_t m = 0;
        for (int l = 0; l < w; l++) m |= (s[l] & 1u) << l;
        return m;
    });
}
template <typename T>
inline T shfl(T v, int src) {
    const int w = width();
    return from_bits<T>(exchange(bits(v), [src, w](const uint64_t *s) {
        return s[((src % w) + w) % w];
    }));
}
template <typename T>
inline T shfl_xor(T v, int m) {
    const int l = lane(), w = width();
    return from_bits<T>(exchange(bits(v), [l, m, w](const uint64_t *s) {
        const int j = l ^ m;
        return s[j < w ? j : l];
    }));
}
inline uint32_t readlane(uint32_t v, int src) {
    return (uint32_t)exchange(v, [src](const uint64_t *s) { return s[src]; });
}
inline uint32_t readfirstlane(uint32_t v) {
    return (uint32_t)exchange(v, [](const uint64_t *s) { return s[0]; });
}
// DPP moves used by the kernels: row_shr:1..15 (0x111..0x11f), row_bcast:15
// (0x142) and row_bcast:31 (0x143); lanes without a valid source, or in rows
// outside row_mask, keep `old` (bound_ctrl off).
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    if (bank_mask != 0xf || bound_ctrl) {
        fprintf(stderr, "emu: unsupported DPP bank mask / bound control\n");
        abort();
    }
    const int l = lane();
    return (int)(uint32_t)exchange((uint32_t)src, [=](const uint64_t *s) -> uint64_t {
        const int row = l >> 4, i = l & 15;
        if (!((row_mask >> row) & 1)) return (uint32_t)old;
        int from = -1;
        if (ctrl >= 0x111 && ctrl <= 0x11f) {
            const int sh = ctrl - 0x110;
            if (i >= sh) from = l - sh;
        } else if (ctrl == 0x142) {
            if (row >= 1) from = 16 * row - 1;
        } else if (ctrl == 0x143) {
            if (row >= 2) from = 31;
        } else {
            fprintf(stderr, "emu: unsupported DPP control 0x%x\n", ctrl);
            abort();
        }
        return from < 0 ? (uint64_t)(uint32_t)old : (uint64_t)(uint32_t)s[from];
    });
}

}  // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::g_block_idx)
#define blockDim (emu::g_dim)
#define gridDim (emu::g_grid)

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
    emu::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)

inline void __syncthreads() { emu::block_barrier(); }
inline int __lane_id() { return emu::lane(); }
inline uint64_t __ballot(int p) { return emu::ballot(p != 0); }
template <typename T> inline T __shfl(T v, int src, int = 64) { return emu::shfl(v, src); }
template <typename T> inline T __shfl_xor(T v, int m, int = 64) { return emu::shfl_xor(v, m); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __clzll(long long v) { return v == 0 ? 64 : __builtin_clzll((unsigned long long)v); }
inline long long __double_as_longlong(double d) { return emu::from_bits<long long>(emu::bits(d)); }
inline double __longlong_as_double(long long v) { return emu::from_bits<double>(emu::bits(v)); }
#define __builtin_amdgcn_readlane(v, l) emu::readlane((uint32_t)(v), (l))
#define __builtin_amdgcn_readfirstlane(v) emu::readfirstlane((uint32_t)(v))
#define __builtin_amdgcn_update_dpp(o, s, c, r, b, bc) emu::update_dpp((o), (s), (c), (r), (b), (bc))
#define __builtin_amdgcn_rsqf(x) (1.0f / sqrtf(x))
#define __builtin_amdgcn_sqrtf(x) sqrtf(x)

template <typename T, typename U> inline T atomicAdd(T *p, U v) {
    return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U> inline T atomicOr(T *p, U v) {
    return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST);
}
template <typename T, typename U> inline T atomicMax(T *p, U v) {
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (old < (T)v && !__atomic_compare_exchange_n(p, &old, (T)v, false, __ATOMIC_SEQ_CST,
                                                      __ATOMIC_SEQ_CST)) {
    }
    return old;
}

extern "C" __attribute__((weak, used)) void emu_fiber_main(emu::Fiber *f) {
    (*emu::g_job)(f->tid);
    emu::yield(emu::FS::done);
    abort();   // a finished fiber is never resumed
}

// ---- runtime -------------------------------------------------------------
typedef enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 } hipError_t;
typedef enum {
    hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4
} hipMemcpyKind;
typedef enum { hipDeviceAttributeMultiprocessorCount = 1 } hipDeviceAttribute_t;
typedef struct emu_stream *hipStream_t;
typedef struct emu_event {
    double t;
} *hipEvent_t;
#define hipEventDisableTiming 2u

inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "error"; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) {
    *v = 1;
    return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    if (n) memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(d, s, n, k);
}
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
    memset(d, v, n);
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new emu_event{0.0};
    return hipSuccess;
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->t = std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
    return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    *ms = (float)(b->t - a->t);
    return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned = 0) {
    *p = calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
// device symbols are ordinary host objects in the emulation
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}
inline hipError_t hipHostFree(void *p) {
    free(p);
    return hipSuccess;
}
