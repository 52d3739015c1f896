// Task bodies (device code).  Each body is a __device__ function run by one
// 256-thread workgroup for one piece; the standalone kernels (in-order and
// plain paths) and the persistent kernel's workers call the same functions,
// so every path computes the same bits.
//
// Floating point: built with -ffp-contract=off and correctly rounded FP32
// division and square root; fused multiply-adds appear only where the task
// definition says fma.  Every reduction has a fixed order defined by the data
// size, never by the number of pieces or workgroups.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "acs_tasks.h"
#include "rl_layout.hpp"

namespace acs {

// Global memory accesses go through pointers in the global address space.
// A pointer the compiler cannot place (one loaded from a struct, or made
// from an integer) is otherwise accessed with FLAT instructions, which count
// on the LDS counter as well: every later wait for an LDS read would then
// also wait for those loads and stores to complete, including device-scope
// stores that travel to memory.  The CPU build of this source has no
// address spaces.
#if defined(__HIP_DEVICE_COMPILE__)
#define ACS_GAS __attribute__((address_space(1)))
#else
#define ACS_GAS
#endif
template <class T>
__device__ __forceinline__ ACS_GAS T *gp(T *p)
{
    return (ACS_GAS T *)p;
}

// 16-byte loads of the vector types through global pointers (their class
// types cannot bind a reference to an object in another address space)
typedef float acs_f4v __attribute__((ext_vector_type(4)));
typedef uint32_t acs_u4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(const ACS_GAS float4 *p)
{
    const acs_f4v v = *reinterpret_cast<const ACS_GAS acs_f4v *>(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 ld4(const ACS_GAS uint4 *p)
{
    const acs_u4v v = *reinterpret_cast<const ACS_GAS acs_u4v *>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// LDS scratch every body may use (bytes).
constexpr int kBodySmem = 40 * 1024;

__device__ inline void piece_range(uint32_t n, uint32_t piece, uint32_t np, uint32_t &lo, uint32_t &hi)
{
    uint32_t per = (n + np - 1) / np;
    per = (per + 255u) & ~255u;
    lo = piece * per;
    hi = lo + per < n ? lo + per : n;
    if (lo > n) lo = n;
}

// Stores of task results.  A standalone kernel stores them plainly: the
// end of the kernel makes them visible to whatever runs next.  Inside the
// persistent kernel (DEV) a piece's results must be visible, as soon as the
// piece is counted, to pieces of other kernels, which may run on another
// XCD with its own L2.  They are stored with device scope, which writes them
// through the L2 of the storing XCD, so that counting a piece only waits for
// its own stores instead of writing back that whole L2.  Host memory (the
// island plan) is stored with system scope.  The device-scope stores are
// integer stores of the same bits (a 16-byte value as two 8-byte halves).
template <bool DEV>
__device__ __forceinline__ void put(ACS_GAS int32_t *p, int32_t v)
{
    if constexpr (DEV) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <bool DEV>
__device__ __forceinline__ void put(ACS_GAS float *p, float v)
{
    if constexpr (DEV)
        __hip_atomic_store(reinterpret_cast<ACS_GAS uint32_t *>(p), (uint32_t)__float_as_uint(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <bool DEV, typename V16>
__device__ __forceinline__ void put16(ACS_GAS V16 *p, const V16 &v)
{
    static_assert(sizeof(V16) == 16, "16-byte value");
    if constexpr (DEV) {
        uint64_t h[2];
        __builtin_memcpy(h, &v, 16);
        ACS_GAS uint64_t *q = reinterpret_cast<ACS_GAS uint64_t *>(p);
        __hip_atomic_store(q, h[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(q + 1, h[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        *p = v;
    }
}

// Words the host reads while the kernel may still be running (the island
// plan): system-scope stores, written through to host memory, on every path.
__device__ __forceinline__ void put_host(ACS_GAS int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The island plan on its way to the host.  Standalone kernels store it to
// host memory as they compute it.  In the persistent kernel the islands body
// leaves it in LDS, at the end of the body scratch (`plan_stage`), and the
// worker copies it out after it has marked the kernel complete: a store to
// host memory takes from a microsecond to tens of microseconds to complete,
// and no task on the device reads the plan (only the host does, after the
// stamp), so the kernel's dependents need not wait for it.
__device__ __forceinline__ int32_t *plan_stage(uint8_t *smem, int32_t n)
{
    return reinterpret_cast<int32_t *>(smem + kBodySmem) - rl_plan_ints(n);
}

template <bool DEV>
__device__ __forceinline__ void plan_put(ACS_GAS int32_t *plan, int32_t *stage, int32_t i, int32_t v)
{
    if constexpr (DEV)
        stage[i] = v;
    else
        put_host(&plan[i], v);
}

// Copies a staged plan to host memory, the stamp last once the rest has
// completed (whole workgroup; the worker calls it after the completion store).
__device__ inline void plan_publish(const acs_args_rl &a, uint8_t *smem)
{
    ACS_GAS int32_t *plan = reinterpret_cast<ACS_GAS int32_t *>(a.plan);
    const int32_t *stage = plan_stage(smem, a.n);
    const int32_t nm = stage[1];
    const int32_t cnt = 4 + 4 * (nm < 0 ? 0 : (nm > a.n / 2 ? a.n / 2 : nm));
    for (int32_t i = (int32_t)threadIdx.x; i < cnt; i += ACS_BLOCK)
        if (i != 3) put_host(&plan[i], stage[i]);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt 0, expcnt 7, lgkmcnt 15
    __syncthreads();
    if (threadIdx.x == 0) put_host(&plan[3], stage[3]);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// no-op with an optional busy wait on the constant wall clock
// ---------------------------------------------------------------------------
__device__ inline void body_nop(const acs_args_nop &a)
{
    // every wave waits on its own (uniform loop, no lane divergence);
    // wall_clock64 runs at 100 MHz: 10 ns per tick
    if (a.spin_ns != 0) {
        const uint64_t t0 = wall_clock64(), ticks = a.spin_ns / 10;
        while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(1);
    }
}

// ---------------------------------------------------------------------------
// tiny random stream
// ---------------------------------------------------------------------------
template <bool DEV>
__device__ inline void body_scale(const acs_args_scale &a, uint32_t piece, uint32_t np)
{
    uint32_t lo, hi;
    piece_range(a.n, piece, np, lo, hi);
    const ACS_GAS float *x = gp(a.x);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += ACS_BLOCK) put<DEV>(gp(a.out) + i, a.a * x[i]);
}

template <bool DEV>
__device__ inline void body_axpy(const acs_args_axpy &a, uint32_t piece, uint32_t np)
{
    uint32_t lo, hi;
    piece_range(a.n, piece, np, lo, hi);
    const ACS_GAS float *x = gp(a.x), *y = gp(a.y);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += ACS_BLOCK) put<DEV>(gp(a.out) + i, fmaf(a.a, x[i], y[i]));
}

__device__ inline float sum_leaf(const acs_args_sum &a, uint32_t g)
{
    const uint32_t l0 = a.len[0], l1 = a.nin > 1 ? a.len[1] : 0, l2 = a.nin > 2 ? a.len[2] : 0;
    if (g < l0) return gp(a.in[0])[g];
    g -= l0;
    if (g < l1) return gp(a.in[1])[g];
    g -= l1;
    if (g < l2) return gp(a.in[2])[g];
    return 0.0f;
}

constexpr uint32_t kSumMax = 256 * 64;

// Pairwise tree over the zero-padded concatenation (length P, a power of two).
// For the levels s >= 256 the pairs (i, i+s) share i mod 256, so thread t runs
// those levels in registers over its leaves t + 256m; the last eight levels
// run across threads in LDS.  Same additions, same order, as the definition.
template <bool DEV>
__device__ inline void body_sum(const acs_args_sum &a, float *red)
{
    const uint32_t t = threadIdx.x;
    uint32_t T = a.len[0] + (a.nin > 1 ? a.len[1] : 0) + (a.nin > 2 ? a.len[2] : 0);
    uint32_t P = 1;
    while (P < T) P <<= 1;
    uint32_t level;
    if (P >= 256) {
        const uint32_t M = P / 256;
        float v[64];
#pragma unroll
        for (int m = 0; m < 64; m++) v[m] = ((uint32_t)m < M) ? sum_leaf(a, t + 256u * m) : 0.0f;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
            if ((uint32_t)s < M) {
#pragma unroll
                for (int m = 0; m < s; m++) v[m] = v[m] + v[m + s];
            }
        }
        red[t] = v[0];
        level = 128;
    } else {
        red[t] = (t < P) ? sum_leaf(a, t) : 0.0f;
        level = P / 2;
    }
    __syncthreads();
    for (uint32_t s = level; s >= 1; s >>= 1) {
        if (t < s) red[t] = red[t] + red[t + s];
        __syncthreads();
    }
    if (t == 0) put<DEV>(gp(a.out), red[0]);
}

// ---------------------------------------------------------------------------
// rigid-body RL step
// ---------------------------------------------------------------------------
struct RLView {
    ACS_GAS float4 *X, *V, *P, *Q0, *Q1;
    ACS_GAS int32_t *deg, *adj_off, *adj, *label, *perm, *inv_perm, *isl_off, *padj_off, *padj;
};

__device__ inline RLView rl_view(uint64_t base, int32_t n)
{
    uint64_t off[ACS_RL_NREGIONS];
    rl_offsets(n, off);
    ACS_GAS char *b = reinterpret_cast<ACS_GAS char *>(base);
    RLView v;
    v.X = reinterpret_cast<ACS_GAS float4 *>(b + off[ACS_RL_X]);
    v.V = reinterpret_cast<ACS_GAS float4 *>(b + off[ACS_RL_V]);
    v.P = reinterpret_cast<ACS_GAS float4 *>(b + off[ACS_RL_P]);
    v.Q0 = reinterpret_cast<ACS_GAS float4 *>(b + off[ACS_RL_Q0]);
    v.Q1 = reinterpret_cast<ACS_GAS float4 *>(b + off[ACS_RL_Q1]);
    v.deg = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_DEG]);
    v.adj_off = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_ADJ_OFF]);
    v.adj = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_ADJ]);
    v.label = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_LABEL]);
    v.perm = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_PERM]);
    v.inv_perm = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_INV_PERM]);
    v.isl_off = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_ISL_OFF]);
    v.padj_off = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_PADJ_OFF]);
    v.padj = reinterpret_cast<ACS_GAS int32_t *>(b + off[ACS_RL_PADJ]);
    return v;
}

__device__ inline float dist2(float dx, float dy, float dz) { return fmaf(dz, dz, fmaf(dy, dy, dx * dx)); }

// Inclusive prefix sum over a wave's 64 lanes: a scan inside each row of 16
// lanes by DPP row shifts (a lane whose source would leave the row adds 0),
// then the total of row 0 added to rows 1 and 3 (row_bcast:15) and that of
// rows 0-1 to rows 2 and 3 (row_bcast:31).
__device__ inline int32_t wave_inclusive_scan(int32_t x)
{
    int32_t inc = x;
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x111, 0xf, 0xf, false);   // row_shr:1
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x112, 0xf, 0xf, false);   // row_shr:2
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x114, 0xf, 0xf, false);   // row_shr:4
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x118, 0xf, 0xf, false);   // row_shr:8
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x142, 0xa, 0xf, false);   // row_bcast:15
    inc += __builtin_amdgcn_update_dpp(0, inc, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return inc;
}

// Exclusive scan of data[0..n) in place; returns the total.  Thread t sums a
// contiguous chunk; the 256 chunk sums are scanned inside each wave with
// DPP and across the four waves through tmp (4 ints).  Integer only, so
// the grouping does not change the result.
__device__ inline int32_t block_exclusive_scan(int32_t *data, int32_t n, int32_t *tmp)
{
    const int32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int32_t per = (n + ACS_BLOCK - 1) / ACS_BLOCK;
    const int32_t lo = t * per < n ? t * per : n, hi = lo + per < n ? lo + per : n;
    int32_t s = 0;
    for (int32_t i = lo; i < hi; i++) s += data[i];
    const int32_t x = wave_inclusive_scan(s);
    if (lane == 63) tmp[wv] = x;
    __syncthreads();
    int32_t woff = 0;
    for (int k = 0; k < wv; k++) woff += tmp[k];
    const int32_t total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
    int32_t run = woff + x - s;
    for (int32_t i = lo; i < hi; i++) {
        const int32_t v = data[i];
        data[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// Wave-level helpers for scenes of at most 64 bodies (one lane per body).
// The wave index comes from readfirstlane so that branches on it are uniform
// to the compiler as well.
__device__ inline int32_t wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ inline uint64_t lane_read64(uint64_t x, int32_t l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline float lane_readf(float x, int32_t l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); }

// exclusive prefix sum over the wave's lanes in lane order; *total = sum of all
__device__ inline int32_t wave_exclusive_scan(int32_t x, int32_t *total)
{
    const int32_t inc = wave_inclusive_scan(x);
    *total = __builtin_amdgcn_readlane(inc, 63);
    return inc - x;
}

template <bool DEV>
__device__ inline void body_rl_predict(const acs_args_rl &a, uint32_t piece, uint32_t np)
{
    RLView v = rl_view(a.base, a.n);
    uint32_t lo, hi;
    piece_range((uint32_t)a.n, piece, np, lo, hi);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += ACS_BLOCK) {
        float4 x = ld4(&v.X[i]), u = ld4(&v.V[i]), p;
        p.x = fmaf(a.dt, u.x, x.x);
        p.y = fmaf(a.dt, u.y, x.y);
        p.z = fmaf(a.dt, u.z, x.z);
        p.w = fmaf(a.dt, u.w, x.w);
        put16<DEV>(&v.P[i], p);
    }
}

// Contacts of every body, adjacency in ascending partner order (CSR).  With
// n <= 128 each body's partners are split into Q = 256 / n contiguous chunks,
// one thread per (body, chunk), so that every thread of the workgroup works;
// chunk counts give each thread its write position, which keeps the
// adjacency in partner order.
// At most 64 bodies: lane i holds body i in every wave; wave w tests the
// partners j = w, w + 4, ... against all bodies at once, and the ballot of the
// contact test is body j's neighbour set (the test is symmetric bit for bit:
// the differences only change sign).  Wave 0 then writes degrees, offsets and
// the adjacency in ascending partner order.
template <bool DEV>
__device__ inline void broadphase_small(const acs_args_rl &a, const RLView &v, uint8_t *smem)
{
    const int32_t n = a.n, lane = threadIdx.x & 63, wv = wave_index();
    uint64_t *rows = reinterpret_cast<uint64_t *>(smem);   // [64]
    const bool in = lane < n;
    const float4 pi = in ? ld4(&v.P[lane]) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float two_r = 2.0f * a.r, thr = two_r * two_r;
    for (int32_t j = wv; j < n; j += 4) {
        const float xj = lane_readf(pi.x, j), yj = lane_readf(pi.y, j), zj = lane_readf(pi.z, j);
        const bool hit = in && lane != j && dist2(pi.x - xj, pi.y - yj, pi.z - zj) < thr;
        const uint64_t row = __builtin_amdgcn_ballot_w64(hit);
        if (lane == 0) rows[j] = row;
    }
    __syncthreads();
    if (wv != 0) return;
    const uint64_t mine = in ? rows[lane] : 0ull;
    const int32_t deg = __builtin_popcountll(mine);
    int32_t total;
    const int32_t off = wave_exclusive_scan(deg, &total);
    if (in) {
        put<DEV>(&v.deg[lane], deg);
        put<DEV>(&v.adj_off[lane], off);
    }
    if (lane == 0) put<DEV>(&v.adj_off[n], total);
    int32_t k = off;
    for (uint64_t m = mine; m; m &= m - 1) put<DEV>(&v.adj[k++], (int32_t)__builtin_ctzll(m));
}

template <bool DEV>
__device__ inline void body_rl_broadphase(const acs_args_rl &a, uint8_t *smem)
{
    const int32_t n = a.n, t = threadIdx.x;
    RLView v = rl_view(a.base, n);
    if (n <= 64) {
        broadphase_small<DEV>(a, v, smem);
        return;
    }
    float4 *Ps = reinterpret_cast<float4 *>(smem);                 // 16 n bytes
    int32_t *cnt = reinterpret_cast<int32_t *>(smem + 16 * n);     // max(n, 256) ints
    int32_t *deg = cnt + (n > ACS_BLOCK ? n : ACS_BLOCK);          // n ints
    int32_t *tmp = deg + n;                                        // 4 ints
    for (int32_t i = t; i < n; i += ACS_BLOCK) Ps[i] = ld4(&v.P[i]);
    __syncthreads();
    const float two_r = 2.0f * a.r, thr = two_r * two_r;
    const int32_t Q = n <= 128 ? ACS_BLOCK / n : 1;   // chunks per body
    const int32_t chunk = (n + Q - 1) / Q;
    if (Q > 1) {
        // cnt[q * n + i]: contacts of body i among partners [q*chunk, (q+1)*chunk)
        const int32_t i = t % n, q = t / n;
        if (q < Q) {
            const float4 pi = Ps[i];
            const int32_t j0 = q * chunk, j1 = j0 + chunk < n ? j0 + chunk : n;
            int32_t c = 0;
            for (int32_t j = j0; j < j1; j++) {
                const float4 pj = Ps[j];
                c += (j != i && dist2(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < thr) ? 1 : 0;
            }
            cnt[q * n + i] = c;
        }
        __syncthreads();
        for (int32_t b = t; b < n; b += ACS_BLOCK) {
            int32_t d = 0;
            for (int32_t q2 = 0; q2 < Q; q2++) d += cnt[q2 * n + b];
            deg[b] = d;
            put<DEV>(&v.deg[b], d);
        }
        __syncthreads();
        const int32_t total = block_exclusive_scan(deg, n, tmp);
        if (q < Q) {
            const float4 pi = Ps[i];
            int32_t k = deg[i];
            for (int32_t q2 = 0; q2 < q; q2++) k += cnt[q2 * n + i];
            if (q == 0) put<DEV>(&v.adj_off[i], deg[i]);
            const int32_t j0 = q * chunk, j1 = j0 + chunk < n ? j0 + chunk : n;
            for (int32_t j = j0; j < j1; j++) {
                const float4 pj = Ps[j];
                if (j != i && dist2(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < thr) put<DEV>(&v.adj[k++], j);
            }
        }
        if (t == 0) put<DEV>(&v.adj_off[n], total);
        return;
    }
    // Above 128 bodies: a uniform grid of cells a little wider than 2r (at
    // most 12 per axis), so that a body's contacts lie in its own cell or
    // the 26 around it (cell coordinates are clamped to the grid, which
    // keeps two positions within 2r in neighbouring cells).  The contact
    // test is the same expression as everywhere, so the contact set is the
    // all-pairs one; each body's list is sorted into index order in LDS.
    // Bodies whose lists do not fit in LDS go through the all-pairs walk.
    const float cs = two_r * 1.0009765625f;
    const float inv_cs = 1.0f / cs;
    const int32_t C = (cs > 0.0f && inv_cs >= 1.0f) ? (inv_cs >= 12.0f ? 12 : (int32_t)inv_cs) : 1;
    const int32_t NC = C * C * C;
    int32_t *cstart = tmp + 4;            // NC + 1: bodies of cell c at sorted[cstart[c], cstart[c + 1])
    int32_t *sorted = cstart + NC + 1;    // n
    int32_t *cellof = sorted + n;         // n
    int32_t *ladj = cellof + n;           // the sorted lists, while they fit
    const int32_t lcap = (int32_t)(kBodySmem / 4) - (int32_t)(ladj - reinterpret_cast<int32_t *>(smem));
    auto cell1 = [&](float x) -> int32_t {
        const float f = fminf(fmaxf(x * inv_cs, 0.0f), (float)(C - 1));
        return (int32_t)f;
    };
    for (int32_t c = t; c <= NC; c += ACS_BLOCK) cstart[c] = 0;
    __syncthreads();
    for (int32_t i = t; i < n; i += ACS_BLOCK) {
        const float4 p = Ps[i];
        const int32_t c = cell1(p.x) + C * (cell1(p.y) + C * cell1(p.z));
        cellof[i] = c;
        atomicAdd(&cstart[c], 1);
    }
    __syncthreads();
    block_exclusive_scan(cstart, NC + 1, tmp);
    // cstart[c] is now where cell c starts; place the bodies, then cstart[c]
    // has moved to where cell c ends, which is where cell c + 1 starts
    for (int32_t i = t; i < n; i += ACS_BLOCK) sorted[atomicAdd(&cstart[cellof[i]], 1)] = i;
    __syncthreads();
    // walks every partner of body i in the 27 cells around it
    auto each_partner = [&](int32_t i, auto &&fn) {
        const float4 pi = Ps[i];
        const int32_t c = cellof[i], cx = c % C, cy = (c / C) % C, cz = c / (C * C);
        for (int32_t z = (cz > 0 ? cz - 1 : 0); z <= (cz < C - 1 ? cz + 1 : C - 1); z++)
            for (int32_t y = (cy > 0 ? cy - 1 : 0); y <= (cy < C - 1 ? cy + 1 : C - 1); y++) {
                const int32_t row = C * (y + C * z);
                const int32_t x0 = cx > 0 ? cx - 1 : 0, x1 = cx < C - 1 ? cx + 1 : C - 1;
                // cells x0..x1 of this row are contiguous in the sorted order
                const int32_t k0 = row + x0 == 0 ? 0 : cstart[row + x0 - 1], k1 = cstart[row + x1];
                for (int32_t k = k0; k < k1; k++) {
                    const int32_t j = sorted[k];
                    const float4 pj = Ps[j];
                    if (j != i && dist2(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < thr) fn(j);
                }
            }
    };
    for (int32_t i = t; i < n; i += ACS_BLOCK) {
        int32_t c = 0;
        each_partner(i, [&](int32_t) { c++; });
        deg[i] = c;
        put<DEV>(&v.deg[i], c);
    }
    __syncthreads();
    const int32_t total = block_exclusive_scan(deg, n, tmp);
    for (int32_t i = t; i < n; i += ACS_BLOCK) put<DEV>(&v.adj_off[i], deg[i]);
    if (t == 0) put<DEV>(&v.adj_off[n], total);
    if (total <= lcap) {
        for (int32_t i = t; i < n; i += ACS_BLOCK) {
            const int32_t o = deg[i];
            int32_t k = o;
            each_partner(i, [&](int32_t j) {
                // insertion into the list so far, kept in index order
                int32_t q = k++;
                while (q > o && ladj[q - 1] > j) {
                    ladj[q] = ladj[q - 1];
                    q--;
                }
                ladj[q] = j;
            });
        }
        __syncthreads();
        for (int32_t k = t; k < total; k += ACS_BLOCK) put<DEV>(&v.adj[k], ladj[k]);
        return;
    }
    // too many contacts for LDS: all partners in index order
    for (int32_t i = t; i < n; i += ACS_BLOCK) {
        const float4 pi = Ps[i];
        int32_t k = deg[i];
        for (int32_t j = 0; j < n; j++) {
            const float4 pj = Ps[j];
            if (j != i && dist2(pi.x - pj.x, pi.y - pj.y, pi.z - pj.z) < thr) put<DEV>(&v.adj[k++], j);
        }
    }
}

// Connected components by min-label propagation (the fixpoint labels every
// body with the smallest body of its component), then islands ordered by that
// smallest body, bodies inside an island in index order, the adjacency in
// permuted positions, and the plan of multi-body islands for the host.
// At most 64 bodies: the workgroup stages the adjacency in LDS, then one
// wave works: neighbour sets as 64-bit masks, each island grown from its
// smallest body by breadth-first steps that are single ballots, its label
// that smallest body.  Positions: islands in label order (each
// island's first position a scan of the sizes over the roots), bodies in
// index order inside an island.
template <bool DEV>
__device__ inline void islands_small(const acs_args_rl &a, const RLView &v, ACS_GAS int32_t *plan, uint8_t *smem)
{
    const int32_t n = a.n, lane = threadIdx.x & 63;
    const bool in = lane < n;
    int32_t *s_perm = reinterpret_cast<int32_t *>(smem);   // [64] body at each position
    int32_t *s_inv = s_perm + 64;                          // [64] position of each body
    int32_t *s_adj = s_inv + 64;                           // [cap] the adjacency, staged
    const int32_t cap = n * (n - 1);
    // the whole workgroup stages the adjacency in LDS with independent
    // loads, so that no lane walks its neighbours through dependent global
    // loads; offsets past the staged part are clamped to it
    int32_t ecount = v.adj_off[n];
    ecount = ecount < 0 ? 0 : (ecount > cap ? cap : ecount);
    for (int32_t k = (int32_t)threadIdx.x; k < ecount; k += 4 * ACS_BLOCK) {
        int32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = k + u * ACS_BLOCK < ecount ? v.adj[k + u * ACS_BLOCK] : 0;
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (k + u * ACS_BLOCK < ecount) s_adj[k + u * ACS_BLOCK] = c[u];
    }
    __syncthreads();
    if (wave_index() != 0) return;
    int32_t o0 = 0, o1 = 0;
    if (in) {
        o0 = v.adj_off[lane];
        o1 = v.adj_off[lane + 1];
        o0 = o0 < 0 ? 0 : (o0 > ecount ? ecount : o0);
        o1 = o1 < o0 ? o0 : (o1 > ecount ? ecount : o1);
    }
    uint64_t reach = in ? (1ull << lane) : 0ull;
    for (int32_t k = o0; k < o1; k++) {
        const int32_t c = s_adj[k];
        if ((uint32_t)c < (uint32_t)n) reach |= 1ull << c;
    }
    // components by breadth-first search on ballots, one island at a time:
    // the island grows by every body with a neighbour in it (contact is
    // symmetric) until it stops growing; a body without neighbours is an
    // island of its own
    const uint64_t nbrs = reach;
    for (uint64_t todo = __builtin_amdgcn_ballot_w64(o1 > o0); todo;) {
        uint64_t f = 1ull << __builtin_ctzll(todo);
        for (;;) {
            const uint64_t g = __builtin_amdgcn_ballot_w64((nbrs & f) != 0ull) | f;
            if (g == f) break;
            f = g;
        }
        if ((f >> lane) & 1ull) reach = f;
        todo &= ~f;
    }
    const int32_t root = in ? __builtin_ctzll(reach) : lane;
    const bool isroot = in && root == lane;
    const uint64_t roots = __builtin_amdgcn_ballot_w64(isroot);
    const int32_t nisl = __builtin_popcountll(roots);
    const int32_t size = __builtin_popcountll(reach);
    // first position of each island: the sizes of the islands with smaller
    // labels, a scan over the roots read back at each body's root
    int32_t nin;
    const int32_t rstart = wave_exclusive_scan(isroot ? size : 0, &nin);
    const int32_t start = __shfl(rstart, root & 63, 64);
    const uint64_t below = (1ull << lane) - 1ull;   // lane 0: empty
    const int32_t pos = start + __builtin_popcountll(reach & below);
    const int32_t ridx = __builtin_popcountll(roots & ((1ull << root) - 1ull));
    if (in) {
        put<DEV>(&v.label[lane], root);
        put<DEV>(&v.perm[pos], lane);
        put<DEV>(&v.inv_perm[lane], pos);
        s_perm[pos] = lane;
        s_inv[lane] = pos;
    }
    if (isroot) put<DEV>(&v.isl_off[ridx], start);
    if (lane == 0) put<DEV>(&v.isl_off[nisl], n);
    // the stores above land before the loads below (one wave, LDS in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t b = in ? s_perm[lane] : 0;           // body at position `lane`
    const int32_t db = __shfl(o1 - o0, b, 64);
    const int32_t ob = __shfl(o0, b, 64);
    int32_t ep;
    const int32_t poff = wave_exclusive_scan(in ? db : 0, &ep);
    if (in) put<DEV>(&v.padj_off[lane], poff);
    if (lane == 0) put<DEV>(&v.padj_off[n], ep);
    // four neighbours at a time, so that their LDS reads overlap
    for (int32_t k = 0; in && k < db; k += 4) {
        int32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = k + u < db ? s_adj[ob + k + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; u++) c[u] = (uint32_t)c[u] < (uint32_t)n ? s_inv[c[u]] : lane;
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (k + u < db && poff + k + u < cap) put<DEV>(&v.padj[poff + k + u], c[u]);
    }
    // plan: multi-body islands in label order
    const bool multi = isroot && size >= 2;
    const uint64_t multis = __builtin_amdgcn_ballot_w64(multi);
    const int32_t e0 = __shfl(poff, start & 63, 64);
    const int32_t endp = start + size;
    const int32_t e1s = __shfl(poff, endp & 63, 64);   // every lane takes part in the shuffle
    const int32_t e1 = endp < n ? e1s : ep;
    int32_t *stage = plan_stage(smem, n);
    if (multi) {
        const int32_t m = __builtin_popcountll(multis & below);
        plan_put<DEV>(plan, stage, 4 + 4 * m + 0, start);
        plan_put<DEV>(plan, stage, 4 + 4 * m + 1, endp);
        plan_put<DEV>(plan, stage, 4 + 4 * m + 2, e0);
        plan_put<DEV>(plan, stage, 4 + 4 * m + 3, e1);
    }
    if (lane == 0) {
        plan_put<DEV>(plan, stage, 0, nisl);
        plan_put<DEV>(plan, stage, 1, (int32_t)__builtin_popcountll(multis));
        plan_put<DEV>(plan, stage, 2, ep);
    }
    if constexpr (DEV) {
        if (lane == 0) stage[3] = a.iter;   // published after completion (plan_publish)
    } else {
        // the stamp last, once this wave's plan stores have completed (the
        // wave wrote the whole plan)
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt 0, expcnt 7, lgkmcnt 15
        if (lane == 0) put_host(&plan[3], a.iter);
    }
}

template <bool DEV>
__device__ inline void body_rl_islands(const acs_args_rl &a, uint8_t *smem)
{
    const int32_t n = a.n, t = threadIdx.x;
    RLView v = rl_view(a.base, n);
    ACS_GAS int32_t *plan = reinterpret_cast<ACS_GAS int32_t *>(a.plan);
    if (n <= 64) {
        islands_small<DEV>(a, v, plan, smem);
        return;
    }
    int32_t *lab = reinterpret_cast<int32_t *>(smem);   // n
    int32_t *aoff = lab + n;                            // n + 1
    int32_t *ridx = aoff + n + 1;                       // n: island index of each root
    int32_t *sz = ridx + n;                             // n + 1: island sizes -> offsets
    int32_t *perm = sz + n + 1;                         // n
    int32_t *inv = perm + n;                            // n
    int32_t *poff = inv + n;                            // n + 1
    int32_t *tmp = poff + n + 1;                        // 4
    int32_t *adjs = tmp + 4;                            // adjacency copy when it fits
    int32_t *stage = plan_stage(smem, n);               // the plan (persistent kernel), at the end
    const int32_t lds_cap = (int32_t)(stage - adjs);

    // offsets are clamped to the adjacency capacity so that a corrupt input
    // can never index outside the arena
    const int32_t cap = n * (n - 1);
    for (int32_t i = t; i <= n; i += ACS_BLOCK) {
        const int32_t o = v.adj_off[i];
        aoff[i] = o < 0 ? 0 : (o > cap ? cap : o);
    }
    for (int32_t i = t; i < n; i += ACS_BLOCK) lab[i] = i;
    __syncthreads();
    // one coalesced copy of the adjacency into LDS instead of dependent
    // global loads inside the propagation loop
    const int32_t E = aoff[n];
    const int32_t *A = (const int32_t *)v.adj;   // global, or the LDS copy below
    if (E <= lds_cap) {
        for (int32_t k = t; k < E; k += ACS_BLOCK) adjs[k] = v.adj[k];
        __syncthreads();
        A = adjs;
    }
    // Connected components by union-find over the contact pairs: a root is
    // only ever hooked under a smaller root (a compare-and-swap on its own
    // label), so each component ends rooted at its smallest body; finds
    // halve their paths, which keeps every label pointing at an ancestor.
    auto ld = [&](int32_t x) { return __hip_atomic_load(&lab[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
    auto find = [&](int32_t x) {
        int32_t p = ld(x);
        while (p != x) {
            const int32_t q = ld(p);
            if (q != p) __hip_atomic_store(&lab[x], q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            x = p;
            p = q;
        }
        return x;
    };
    for (int32_t i = t; i < n; i += ACS_BLOCK)
        for (int32_t k = aoff[i]; k < aoff[i + 1]; k++) {
            const int32_t c = A[k];
            if ((uint32_t)c >= (uint32_t)n || c <= i) continue;   // each pair once; never out of range for broadphase output
            int32_t ri = find(i), rj = find(c);
            while (ri != rj) {
                if (ri > rj) {
                    const int32_t s2 = ri;
                    ri = rj;
                    rj = s2;
                }
                int32_t expect = rj;
                if (__hip_atomic_compare_exchange_strong(&lab[rj], &expect, ri, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                // rj was hooked elsewhere meanwhile: continue from the roots
                ri = find(ri);
                rj = find(expect);
            }
        }
    __syncthreads();
    for (int32_t i = t; i < n; i += ACS_BLOCK) {
        const int32_t r = find(i);
        __hip_atomic_store(&lab[i], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    // island index of each root (roots in ascending order)
    for (int32_t i = t; i < n; i += ACS_BLOCK) ridx[i] = (lab[i] == i) ? 1 : 0;
    __syncthreads();
    const int32_t nisl = block_exclusive_scan(ridx, n, tmp);
    for (int32_t k = t; k <= n; k += ACS_BLOCK) sz[k] = 0;
    __syncthreads();
    for (int32_t i = t; i < n; i += ACS_BLOCK) atomicAdd(&sz[ridx[lab[i]]], 1);
    __syncthreads();
    block_exclusive_scan(sz, nisl, tmp);
    if (t == 0) sz[nisl] = n;
    __syncthreads();
    for (int32_t k = t; k <= nisl; k += ACS_BLOCK) put<DEV>(&v.isl_off[k], sz[k]);
    // Positions: bodies ordered by (label, index), islands in label order and
    // bodies in index order inside each.  A bitonic sort of the keys
    // label * 2048 + index (n <= 1024), padded to a power of two, in the
    // perm and inv arrays (2n entries, at least the padded size).
    int32_t P = 1;
    while (P < n) P <<= 1;
    int32_t *key = perm;
    for (int32_t i = t; i < P; i += ACS_BLOCK) key[i] = i < n ? (lab[i] << 11) | i : 0x7FFFFFFF;
    __syncthreads();
    for (int32_t k = 2; k <= P; k <<= 1)
        for (int32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int32_t i = t; i < P; i += ACS_BLOCK) {
                const int32_t l = i ^ jj;
                if (l > i) {
                    const int32_t a0 = key[i], a1 = key[l];
                    const bool up = (i & k) == 0;
                    if ((a0 > a1) == up) {
                        key[i] = a1;
                        key[l] = a0;
                    }
                }
            }
            __syncthreads();
        }
    // the n real keys sort first and name the body at each position; perm
    // is rewritten in place, inv lands where only padding was
    for (int32_t p = t; p < n; p += ACS_BLOCK) {
        const int32_t i = key[p] & 2047;
        perm[p] = i;
        inv[i] = p;
        put<DEV>(&v.label[i], lab[i]);
        put<DEV>(&v.perm[p], i);
        put<DEV>(&v.inv_perm[i], p);
    }
    __syncthreads();
    for (int32_t p = t; p < n; p += ACS_BLOCK) {
        const int32_t d = aoff[perm[p] + 1] - aoff[perm[p]];
        poff[p] = d > 0 ? d : 0;
    }
    __syncthreads();
    const int32_t Ep = block_exclusive_scan(poff, n, tmp);
    if (t == 0) poff[n] = Ep;
    __syncthreads();
    for (int32_t p = t; p <= n; p += ACS_BLOCK) put<DEV>(&v.padj_off[p], poff[p]);
    for (int32_t p = t; p < n; p += ACS_BLOCK) {
        const int32_t b = perm[p], k0 = aoff[b], d = aoff[b + 1] - k0, o = poff[p];
        for (int32_t k = 0; k < d; k++) {
            const int32_t c = A[k0 + k];
            if (o + k < cap) put<DEV>(&v.padj[o + k], ((uint32_t)c < (uint32_t)n) ? inv[c] : p);
        }
    }
    // plan: multi-body islands in island order (reuse ridx as flags)
    __syncthreads();
    for (int32_t k = t; k < nisl; k += ACS_BLOCK) ridx[k] = (sz[k + 1] - sz[k] >= 2) ? 1 : 0;
    __syncthreads();
    const int32_t nmulti = block_exclusive_scan(ridx, nisl, tmp);
    for (int32_t k = t; k < nisl; k += ACS_BLOCK) {
        if (sz[k + 1] - sz[k] >= 2) {
            const int32_t m = ridx[k];
            plan_put<DEV>(plan, stage, 4 + 4 * m + 0, sz[k]);
            plan_put<DEV>(plan, stage, 4 + 4 * m + 1, sz[k + 1]);
            plan_put<DEV>(plan, stage, 4 + 4 * m + 2, poff[sz[k]]);
            plan_put<DEV>(plan, stage, 4 + 4 * m + 3, poff[sz[k + 1]]);
        }
    }
    if (t == 0) {
        plan_put<DEV>(plan, stage, 0, nisl);
        plan_put<DEV>(plan, stage, 1, nmulti);
        plan_put<DEV>(plan, stage, 2, Ep);
    }
    if constexpr (DEV) {
        if (t == 0) stage[3] = a.iter;   // published after completion (plan_publish)
    } else {
        // the stamp last, once every wave's plan stores have completed
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt 0, expcnt 7, lgkmcnt 15
        __syncthreads();
        if (t == 0) put_host(&plan[3], a.iter);
    }
}

template <bool DEV>
__device__ inline void body_rl_permute(const acs_args_rl &a, uint32_t piece, uint32_t np)
{
    RLView v = rl_view(a.base, a.n);
    uint32_t lo, hi;
    piece_range((uint32_t)a.n, piece, np, lo, hi);
    for (uint32_t p = lo + threadIdx.x; p < hi; p += ACS_BLOCK) {
        const uint32_t b = (uint32_t)v.perm[p];
        put16<DEV>(&v.Q0[p], ld4(&v.P[b < (uint32_t)a.n ? b : p]));
    }
}

// One Jacobi iteration over the island's positions [b0, b1).
template <bool DEV>
__device__ inline void body_rl_jacobi(const acs_args_rl &a)
{
    RLView v = rl_view(a.base, a.n);
    const ACS_GAS float4 *src = (a.iter % 2 == 0) ? v.Q0 : v.Q1;
    ACS_GAS float4 *dst = (a.iter % 2 == 0) ? v.Q1 : v.Q0;
    const float two_r = 2.0f * a.r;
    for (int32_t p = a.b0 + (int32_t)threadIdx.x; p < a.b1; p += ACS_BLOCK) {
        const float4 qp = ld4(&src[p]);
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
        const int32_t cap = a.n * (a.n - 1);
        int32_t e0 = v.padj_off[p], e1 = v.padj_off[p + 1];
        e0 = e0 < 0 ? 0 : (e0 > cap ? cap : e0);
        e1 = e1 < e0 ? e0 : (e1 > cap ? cap : e1);
        for (int32_t e = e0; e < e1; e++) {
            int32_t q = v.padj[e];
            if ((uint32_t)q >= (uint32_t)a.n) q = p;   // never true for islands output
            const float4 qq = ld4(&src[q]);
            const float dx = qp.x - qq.x, dy = qp.y - qq.y, dz = qp.z - qq.z;
            const float d = sqrtf(dist2(dx, dy, dz));
            const float pen = two_r - d;
            if (pen > 0.0f) {
                const float h = 0.5f * pen;
                float nx, ny, nz;
                if (d > 0.0f) {
                    nx = dx / d;
                    ny = dy / d;
                    nz = dz / d;
                } else {
                    nx = (p < q) ? 1.0f : -1.0f;
                    ny = 0.0f;
                    nz = 0.0f;
                }
                ax = fmaf(h, nx, ax);
                ay = fmaf(h, ny, ay);
                az = fmaf(h, nz, az);
            }
        }
        const float deg = (float)(e1 - e0);
        float4 o;
        o.x = qp.x + ax / deg;
        o.y = qp.y + ay / deg;
        o.z = qp.z + az / deg;
        o.w = qp.w;
        put16<DEV>(&dst[p], o);
    }
}

__device__ inline float wall(float x, float &vel, float lo, float hi)
{
    if (x < lo) {
        vel = fabsf(vel);
        return lo;
    }
    if (x > hi) {
        vel = -fabsf(vel);
        return hi;
    }
    return x;
}

template <bool DEV>
__device__ inline void body_rl_integrate(const acs_args_rl &a, uint32_t piece, uint32_t np)
{
    RLView v = rl_view(a.base, a.n);
    uint32_t lo, hi;
    piece_range((uint32_t)a.n, piece, np, lo, hi);
    const float wlo = a.r, whi = 1.0f - a.r;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += ACS_BLOCK) {
        const uint32_t ip = (uint32_t)v.inv_perm[i];
        const float4 q = ld4(&v.Q0[ip < (uint32_t)a.n ? ip : i]), p = ld4(&v.P[i]);
        float4 u = ld4(&v.V[i]), x;
        u.x = u.x + (q.x - p.x) / a.dt;
        u.y = u.y + (q.y - p.y) / a.dt;
        u.z = u.z + (q.z - p.z) / a.dt;
        x.x = wall(q.x, u.x, wlo, whi);
        x.y = wall(q.y, u.y, wlo, whi);
        x.z = wall(q.z, u.z, wlo, whi);
        x.w = q.w;
        put16<DEV>(&v.X[i], x);
        put16<DEV>(&v.V[i], u);
    }
}

// ---------------------------------------------------------------------------
// dispatch by task type
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// dynamic DNN bodies (NHWC, batch 1)
// ---------------------------------------------------------------------------
typedef float acs_v4f __attribute__((ext_vector_type(4)));

constexpr int kConvKC = 32;   // K columns per step of one wave

// Implicit-GEMM convolution: C[M x N] = A[M x K] B[K x N], M = output pixels,
// N = output channels, K = (ky, kx, ci).  One workgroup computes a 16 x 32
// tile, the reduction over K split between its four waves: wave w takes the
// 32-column steps w, w + 4, ... and keeps two 16x16 accumulators of
// v_mfma_f32_16x16x4f32 (A element (i, k) from lane i + 16k, B element (k, j)
// from lane j + 16k, result (4q + r, j) in lane j + 16q, register r).
// Inside a step, the four k lanes of the s-th matrix instruction hold the
// step's channels q * 8 + s (q = lane / 16), so each lane loads its pixel's
// eight channels q * 8 .. q * 8 + 7 as two 16-byte loads and no staging
// through LDS is needed.  Because cin is a multiple of 32, a step never
// straddles two (ky, kx) taps.  Each wave keeps the loads of its next two
// steps in flight while the matrix unit works on the current one.  The four partial tiles meet in LDS
// and are added in wave order, then the bias: the same order on every path
// and for every piece count.
struct ConvStep {
    float4 a0, a1;          // this lane's pixel, channels q * 8 .. q * 8 + 7 of the step
    float b0[8], b1[8];     // rows q * 8 + s of the step, columns n0 + j and n0 + 16 + j
};

__device__ __forceinline__ void conv_load(const acs_args_conv &a, int32_t py, int32_t px, int32_t n0, int32_t kc0,
                                          int32_t q, int32_t j, ConvStep &v)
{
    const int32_t cin = a.cin, k = a.k, st = a.stride, pad = (k - 1) / 2, hin = a.hin, cout = a.cout;
    const int32_t tap = kc0 / cin, ci0 = kc0 - tap * cin, ky = tap / k, kx = tap - ky * k;
    const int32_t iy = py * st + ky - pad, ix = px * st + kx - pad;
    v.a0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    v.a1 = v.a0;
    if (iy >= 0 && iy < hin && ix >= 0 && ix < hin) {
        const ACS_GAS float4 *src = reinterpret_cast<const ACS_GAS float4 *>(gp(a.in) + ((int64_t)iy * hin + ix) * cin + ci0 + q * 8);
        v.a0 = ld4(src);
        v.a1 = ld4(src + 1);
    }
    const ACS_GAS float *wr = gp(a.w) + (int64_t)(kc0 + q * 8) * cout + n0 + j;
#pragma unroll
    for (int s = 0; s < 8; s++) {
        v.b0[s] = wr[(int64_t)s * cout];
        v.b1[s] = wr[(int64_t)s * cout + 16];
    }
}

// one step: eight k of the 16x16 products of both column halves, in k order
__device__ __forceinline__ void conv_mma(const ConvStep &v, acs_v4f &acc0, acs_v4f &acc1)
{
    const float av[8] = {v.a0.x, v.a0.y, v.a0.z, v.a0.w, v.a1.x, v.a1.y, v.a1.z, v.a1.w};
#pragma unroll
    for (int s = 0; s < 8; s++) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], v.b0[s], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], v.b1[s], acc1, 0, 0, 0);
    }
}

template <bool DEV>
__device__ inline void conv_tile(const acs_args_conv &a, int32_t m0, int32_t n0, uint8_t *smem)
{
    const int32_t k = a.k, st = a.stride, pad = (k - 1) / 2, cout = a.cout;
    const int32_t hout = (a.hin + 2 * pad - k) / st + 1;
    const int32_t nsteps = k * k * a.cin / kConvKC;
    const int32_t t = threadIdx.x, lane = t & 63, wv = wave_index();
    const int32_t i = lane & 15, q = lane >> 4;
    const int32_t pm = m0 + i, py = pm / hout, px = pm % hout;
    acs_v4f acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
    // this wave's steps wv, wv + 4, ... with the loads of the next two in
    // flight while one is multiplied (three steps of operands resident)
    ConvStep s0, s1, s2;
    if (wv < nsteps) conv_load(a, py, px, n0, wv * kConvKC, q, i, s0);
    if (wv + 4 < nsteps) conv_load(a, py, px, n0, (wv + 4) * kConvKC, q, i, s1);
    for (int32_t step = wv; step < nsteps; step += 12) {
        if (step + 8 < nsteps) conv_load(a, py, px, n0, (step + 8) * kConvKC, q, i, s2);
        conv_mma(s0, acc0, acc1);
        if (step + 4 >= nsteps) break;
        if (step + 12 < nsteps) conv_load(a, py, px, n0, (step + 12) * kConvKC, q, i, s0);
        conv_mma(s1, acc0, acc1);
        if (step + 8 >= nsteps) break;
        if (step + 16 < nsteps) conv_load(a, py, px, n0, (step + 16) * kConvKC, q, i, s1);
        conv_mma(s2, acc0, acc1);
    }
    // partial tiles: part[w][row][col], 4 x 16 x 32 floats
    float *part = reinterpret_cast<float *>(smem);
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const int32_t row = 4 * q + r;
        part[(wv * 16 + row) * 32 + i] = acc0[r];
        part[(wv * 16 + row) * 32 + 16 + i] = acc1[r];
    }
    __syncthreads();
    // 512 outputs, two per thread: wave order, then the bias
    for (int32_t e = t; e < 16 * 32; e += ACS_BLOCK) {
        const int32_t row = e >> 5, col = e & 31;
        float v = part[row * 32 + col];
        v += part[(16 + row) * 32 + col];
        v += part[(32 + row) * 32 + col];
        v += part[(48 + row) * 32 + col];
        put<DEV>(gp(a.out) + (int64_t)(m0 + row) * cout + n0 + col, v + gp(a.bias)[n0 + col]);
    }
}

// Tiles are dealt to pieces round-robin: each output element is computed by
// one tile in one order, whatever the piece count.
template <bool DEV>
__device__ inline void body_conv(const acs_args_conv &a, uint32_t piece, uint32_t np, uint8_t *smem)
{
    const int32_t pad = (a.k - 1) / 2, hout = (a.hin + 2 * pad - a.k) / a.stride + 1;
    const uint32_t ntn = (uint32_t)a.cout / 32u, ntiles = (uint32_t)(hout * hout / 16) * ntn;
    for (uint32_t tile = piece; tile < ntiles; tile += np) {
        conv_tile<DEV>(a, (int32_t)(tile / ntn) * 16, (int32_t)(tile % ntn) * 32, smem);
        __syncthreads();   // the next tile reuses the partial-tile buffer
    }
}

__device__ inline float relu(float x) { return x > 0.0f ? x : 0.0f; }

// Elementwise; 16-byte accesses where the piece and the buffers allow
// (pieces start on multiples of 256 elements), scalar otherwise.
template <bool DEV>
__device__ inline void body_join(const acs_args_join &a, uint32_t piece, uint32_t np)
{
    uint32_t lo, hi;
    piece_range(a.n, piece, np, lo, hi);
    const bool v4 = ((uintptr_t)a.out | (uintptr_t)a.a | (uintptr_t)(a.b ? a.b : a.a)) % 16 == 0;
    uint32_t i = lo;
    if (v4) {
        const uint32_t hv = lo + (hi - lo) / 4 * 4;
        for (uint32_t q = lo / 4 + threadIdx.x; q < hv / 4; q += ACS_BLOCK) {
            const float4 x = ld4(reinterpret_cast<const ACS_GAS float4 *>(gp(a.a)) + q);
            float4 y = a.b ? ld4(reinterpret_cast<const ACS_GAS float4 *>(gp(a.b)) + q) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float4 r;
            if (a.b) {
                r.x = relu(x.x + y.x);
                r.y = relu(x.y + y.y);
                r.z = relu(x.z + y.z);
                r.w = relu(x.w + y.w);
            } else {
                r.x = relu(x.x);
                r.y = relu(x.y);
                r.z = relu(x.z);
                r.w = relu(x.w);
            }
            put16<DEV>(reinterpret_cast<ACS_GAS float4 *>(gp(a.out)) + q, r);
        }
        i = hv;
    }
    if (a.b) {
        for (uint32_t e = i + threadIdx.x; e < hi; e += ACS_BLOCK) put<DEV>(gp(a.out) + e, relu(gp(a.a)[e] + gp(a.b)[e]));
    } else {
        for (uint32_t e = i + threadIdx.x; e < hi; e += ACS_BLOCK) put<DEV>(gp(a.out) + e, relu(gp(a.a)[e]));
    }
}

// one thread per channel; pixel order, FP32.  The loads of a block of 16
// pixels are issued before its additions, which stay in pixel order.
template <bool DEV>
__device__ inline void body_avgpool(const acs_args_avgpool &a)
{
    for (int32_t c = threadIdx.x; c < a.c; c += ACS_BLOCK) {
        float acc = 0.0f;
        int32_t q = 0;
        for (; q + 16 <= a.hw; q += 16) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; u++) v[u] = gp(a.in)[(int64_t)(q + u) * a.c + c];
#pragma unroll
            for (int u = 0; u < 16; u++) acc += v[u];
        }
        for (; q < a.hw; q++) acc += gp(a.in)[(int64_t)q * a.c + c];
        put<DEV>(gp(a.out) + c, acc / (float)a.hw);
    }
}

// one thread per output; fmaf chain in input order (a GEMV: no matrix unit),
// loads of 16 inputs issued ahead of their part of the chain
template <bool DEV>
__device__ inline void body_fc(const acs_args_fc &a)
{
    for (int32_t j = threadIdx.x; j < a.cout; j += ACS_BLOCK) {
        float acc = gp(a.bias)[j];
        int32_t i = 0;
        for (; i + 16 <= a.cin; i += 16) {
            float x[16], w[16];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                x[u] = gp(a.in)[i + u];
                w[u] = gp(a.w)[(int64_t)(i + u) * a.cout + j];
            }
#pragma unroll
            for (int u = 0; u < 16; u++) acc = fmaf(x[u], w[u], acc);
        }
        for (; i < a.cin; i++) acc = fmaf(gp(a.in)[i], gp(a.w)[(int64_t)i * a.cout + j], acc);
        put<DEV>(gp(a.out) + j, acc);
    }
}

// uint4 copy, pieces take consecutive 4 KiB chunks round-robin
template <bool DEV>
__device__ inline void body_copy(const acs_args_copy &a, uint32_t piece, uint32_t np)
{
    const uint64_t nv = a.bytes / 16;
    const ACS_GAS uint4 *src = reinterpret_cast<const ACS_GAS uint4 *>(gp(a.src));
    ACS_GAS uint4 *dst = reinterpret_cast<ACS_GAS uint4 *>(gp(a.dst));
    for (uint64_t i = (uint64_t)piece * ACS_BLOCK + threadIdx.x; i < nv; i += (uint64_t)np * ACS_BLOCK) put16<DEV>(&dst[i], ld4(&src[i]));
}

// one lane stores; the system-scope release orders it after the writes of
// every kernel this one waited for (written through with device scope and
// counted before this body's worker acquired and started), so the host
// that sees the flag sees their results
__device__ inline void body_signal(const acs_args_signal &a)
{
    if (threadIdx.x == 0) __hip_atomic_store(gp(a.addr), a.value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename T>
__device__ inline T load_args(const void *p)
{
    T a;
    __builtin_memcpy(&a, p, sizeof(T));
    return a;
}

template <bool DEV>
__device__ __forceinline__ void run_body(int32_t kid, const void *args, uint32_t piece, uint32_t np, uint8_t *smem)
{
    switch (kid) {
    case ACS_K_NOP: body_nop(load_args<acs_args_nop>(args)); break;
    case ACS_K_SCALE: body_scale<DEV>(load_args<acs_args_scale>(args), piece, np); break;
    case ACS_K_AXPY: body_axpy<DEV>(load_args<acs_args_axpy>(args), piece, np); break;
    case ACS_K_SUM: body_sum<DEV>(load_args<acs_args_sum>(args), reinterpret_cast<float *>(smem)); break;
    case ACS_K_RL_PREDICT: body_rl_predict<DEV>(load_args<acs_args_rl>(args), piece, np); break;
    case ACS_K_RL_BROADPHASE: body_rl_broadphase<DEV>(load_args<acs_args_rl>(args), smem); break;
    case ACS_K_RL_ISLANDS: body_rl_islands<DEV>(load_args<acs_args_rl>(args), smem); break;
    case ACS_K_RL_PERMUTE: body_rl_permute<DEV>(load_args<acs_args_rl>(args), piece, np); break;
    case ACS_K_RL_JACOBI: body_rl_jacobi<DEV>(load_args<acs_args_rl>(args)); break;
    case ACS_K_RL_INTEGRATE: body_rl_integrate<DEV>(load_args<acs_args_rl>(args), piece, np); break;
    case ACS_K_CONV: body_conv<DEV>(load_args<acs_args_conv>(args), piece, np, smem); break;
    case ACS_K_JOIN: body_join<DEV>(load_args<acs_args_join>(args), piece, np); break;
    case ACS_K_AVGPOOL: body_avgpool<DEV>(load_args<acs_args_avgpool>(args)); break;
    case ACS_K_FC: body_fc<DEV>(load_args<acs_args_fc>(args)); break;
    case ACS_K_COPY: body_copy<DEV>(load_args<acs_args_copy>(args), piece, np); break;
    case ACS_K_SIGNAL: body_signal(load_args<acs_args_signal>(args)); break;
    default: break;
    }
}

}  // namespace acs
