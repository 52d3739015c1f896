// Host emulation of the HIP device built-ins used by the scheduler's device
// code, so that persistent.hpp and bodies.hpp build unchanged for the CPU.
// Every GPU thread is an OS thread; a wavefront is 64 of them.  Ballot and
// readlane are rendezvous of the 64 lanes; __syncthreads is a workgroup
// barrier.  Atomics and fences map to sequentially consistent host atomics,
// which is stronger than the GPU memory model (so the emulation checks the
// scheduler's logic, not its GPU memory ordering).
// Test infrastructure only: never part of libacs.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <barrier>
#include <thread>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __align__(x) alignas(x)

#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __HIP_MEMORY_SCOPE_SYSTEM 4

struct float4 {
    float x, y, z, w;
};
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }
struct uint4 {
    uint32_t x, y, z, w;
};
inline uint4 make_uint4(uint32_t x, uint32_t y, uint32_t z, uint32_t w) { return uint4{x, y, z, w}; }

namespace acs_sim {
struct Dim {
    uint32_t x, y, z;
};
struct Wave {
    std::barrier<> bar{64};
    uint64_t vals[64];
    uint64_t base;
};
struct Group {
    std::barrier<> *bar;
    std::atomic<int> orflag{0};
    Wave waves[4];
};
extern thread_local uint32_t tid, bid;
extern thread_local Group *group;
}  // namespace acs_sim

#define threadIdx (acs_sim::Dim{acs_sim::tid, 0, 0})
#define blockIdx (acs_sim::Dim{acs_sim::bid, 0, 0})

#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
// An atomic add by a whole wave is one read-modify-write of the sum of the
// lanes' values, each lane receiving the old value plus the values of the
// lanes below it (what the device compiler emits for an atomic with a
// wave-uniform address).  A rendezvous of the 64 lanes: only for calls made
// by the whole wave, as the kernel source's are.
template <typename T, typename V>
inline T acs_sim_wave_fetch_add(T *p, V v);
#define __hip_atomic_fetch_add(p, v, order, scope) acs_sim_wave_fetch_add((p), (v))

inline void __builtin_amdgcn_fence(int, const char *) { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::yield(); }
inline void __builtin_amdgcn_s_waitcnt(int) {}

inline uint64_t wall_clock64()
{
    // 100 MHz ticks, like the GPU's constant clock
    return (uint64_t)(std::chrono::duration_cast<std::chrono::nanoseconds>(
                          std::chrono::steady_clock::now().time_since_epoch())
                          .count() /
                      10);
}

inline void __syncthreads() { acs_sim::group->bar->arrive_and_wait(); }

inline int __syncthreads_or(int p)
{
    acs_sim::Group *g = acs_sim::group;
    if (p) g->orflag.store(1);
    g->bar->arrive_and_wait();
    const int r = g->orflag.load();
    g->bar->arrive_and_wait();
    if (acs_sim::tid == 0) g->orflag.store(0);
    g->bar->arrive_and_wait();
    return r;
}

inline uint64_t __ballot(int pred)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    w.vals[acs_sim::tid % 64] = pred ? 1 : 0;
    w.bar.arrive_and_wait();
    uint64_t m = 0;
    for (int l = 0; l < 64; l++)
        if (w.vals[l]) m |= 1ull << l;
    w.bar.arrive_and_wait();
    return m;
}

inline uint64_t __builtin_amdgcn_ballot_w64(bool pred) { return __ballot(pred ? 1 : 0); }

template <typename T, typename V>
inline T acs_sim_wave_fetch_add(T *p, V v)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    const uint32_t lane = acs_sim::tid % 64;
    w.vals[lane] = (uint64_t)(T)v;
    w.bar.arrive_and_wait();
    if (lane == 0) {
        T sum = 0;
        for (int l = 0; l < 64; l++) sum = (T)(sum + (T)w.vals[l]);
        w.base = (uint64_t)__atomic_fetch_add(p, sum, __ATOMIC_SEQ_CST);
    }
    w.bar.arrive_and_wait();
    T r = (T)w.base;
    for (uint32_t l = 0; l < lane; l++) r = (T)(r + (T)w.vals[l]);
    w.bar.arrive_and_wait();
    return r;
}

// int result, as the device built-in: a caller that widens it without a cast
// sign-extends, exactly as on the GPU
inline int __builtin_amdgcn_readlane(int v, int l)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    w.vals[acs_sim::tid % 64] = (uint32_t)v;
    w.bar.arrive_and_wait();
    const int r = (int)(uint32_t)w.vals[l];
    w.bar.arrive_and_wait();
    return r;
}

// 16x16x4 FP32 matrix step: lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16) and holds C(4 (l / 16) + r, l % 16) in element r.
typedef float acs_sim_v4f __attribute__((ext_vector_type(4)));
inline acs_sim_v4f __builtin_amdgcn_mfma_f32_16x16x4f32(float a, float b, acs_sim_v4f c, int, int, int)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    const uint32_t lane = acs_sim::tid % 64;
    uint32_t ab[2];
    memcpy(&ab[0], &a, 4);
    memcpy(&ab[1], &b, 4);
    w.vals[lane] = ((uint64_t)ab[1] << 32) | ab[0];
    w.bar.arrive_and_wait();
    acs_sim_v4f d = c;
    for (int r = 0; r < 4; r++) {
        const uint32_t i = 4 * (lane / 16) + r, j = lane % 16;
        float acc = 0.0f;
        for (uint32_t k = 0; k < 4; k++) {
            const uint32_t la = i + 16 * k, lb = j + 16 * k;
            const uint32_t ua = (uint32_t)w.vals[la], ub = (uint32_t)(w.vals[lb] >> 32);
            float fa, fb;
            memcpy(&fa, &ua, 4);
            memcpy(&fb, &ub, 4);
            acc += fa * fb;
        }
        d[r] += acc;
    }
    w.bar.arrive_and_wait();
    return d;
}

// DPP move with the controls the device code uses: row_shr:1-15 and
// row_bcast:15 / row_bcast:31.  A lane of a row or bank masked off, or whose
// source is not valid (bound_ctrl false), keeps `old`.
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    const int lane = (int)(acs_sim::tid % 64), row = lane / 16, col = lane % 16;
    w.vals[lane] = (uint32_t)src;
    w.bar.arrive_and_wait();
    int from = -1;
    if (ctrl >= 0x111 && ctrl <= 0x11f) {
        const int k = ctrl - 0x110;
        if (col >= k) from = lane - k;
    } else if (ctrl == 0x142) {
        if (row >= 1) from = 16 * row - 1;
    } else if (ctrl == 0x143) {
        if (row >= 2) from = 31;
    } else {
        abort();
    }
    int r = old;
    if (((row_mask >> row) & 1) && ((bank_mask >> (col / 4)) & 1))
        r = from >= 0 ? (int)(uint32_t)w.vals[from] : (bound_ctrl ? 0 : old);
    w.bar.arrive_and_wait();
    return r;
}

inline void __builtin_amdgcn_wave_barrier() { acs_sim::group->waves[acs_sim::tid / 64].bar.arrive_and_wait(); }

inline int __builtin_amdgcn_readfirstlane(int v)
{
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    w.vals[acs_sim::tid % 64] = (uint32_t)v;
    w.bar.arrive_and_wait();
    const int r = (int)(uint32_t)w.vals[0];
    w.bar.arrive_and_wait();
    return r;
}

inline int __shfl(int v, int src, int width)
{
    (void)width;
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    const uint32_t lane = acs_sim::tid % 64;
    w.vals[lane] = (uint32_t)v;
    w.bar.arrive_and_wait();
    const int r = (int)(uint32_t)w.vals[(uint32_t)src & 63u];
    w.bar.arrive_and_wait();
    return r;
}

inline int __float_as_int(float x)
{
    int r;
    memcpy(&r, &x, 4);
    return r;
}

inline float __int_as_float(int x)
{
    float r;
    memcpy(&r, &x, 4);
    return r;
}

inline unsigned __float_as_uint(float x)
{
    unsigned r;
    memcpy(&r, &x, 4);
    return r;
}

inline int __shfl_up(int v, unsigned d, int width)
{
    (void)width;
    acs_sim::Wave &w = acs_sim::group->waves[acs_sim::tid / 64];
    const uint32_t lane = acs_sim::tid % 64;
    w.vals[lane] = (uint32_t)v;
    w.bar.arrive_and_wait();
    const int r = lane >= d ? (int)(uint32_t)w.vals[lane - d] : v;
    w.bar.arrive_and_wait();
    return r;
}

inline int atomicAdd(int *p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v)
{
    unsigned long long o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return o;
}

inline unsigned long long atomicMax(unsigned long long *p, unsigned long long v)
{
    unsigned long long o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v > o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return o;
}
