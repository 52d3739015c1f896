// Device code: standalone task kernels (in-order and plain paths) and the
// persistent scheduler kernel (device-resident path; its waves are in
// persistent.hpp).
#include <hip/hip_runtime.h>

#include "bodies.hpp"
#include "dev_shared.hpp"
#include "launch.hpp"
#include "persistent.hpp"

namespace acs {

// ---------------------------------------------------------------------------
// standalone kernels (one per task type)
// ---------------------------------------------------------------------------
template <int KID>
constexpr int smem_bytes()
{
    return (KID == ACS_K_SUM) ? 1024
           : (KID == ACS_K_RL_BROADPHASE || KID == ACS_K_RL_ISLANDS) ? kBodySmem
           : (KID == ACS_K_CONV) ? 4 * 16 * 32 * 4
                                 : 16;
}

template <int KID, typename A>
__global__ __launch_bounds__(ACS_BLOCK) void k_task(A a, uint32_t npieces)
{
    __shared__ __align__(16) uint8_t smem[smem_bytes<KID>()];
    run_body<false>(KID, &a, blockIdx.x, npieces, smem);
}

static const void *const k_table[ACS_K_COUNT] = {
    reinterpret_cast<const void *>(&k_task<ACS_K_NOP, acs_args_nop>),
    reinterpret_cast<const void *>(&k_task<ACS_K_SCALE, acs_args_scale>),
    reinterpret_cast<const void *>(&k_task<ACS_K_AXPY, acs_args_axpy>),
    reinterpret_cast<const void *>(&k_task<ACS_K_SUM, acs_args_sum>),
    nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_PREDICT, acs_args_rl>),
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_BROADPHASE, acs_args_rl>),
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_ISLANDS, acs_args_rl>),
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_PERMUTE, acs_args_rl>),
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_JACOBI, acs_args_rl>),
    reinterpret_cast<const void *>(&k_task<ACS_K_RL_INTEGRATE, acs_args_rl>),
    nullptr, nullptr, nullptr, nullptr,
    reinterpret_cast<const void *>(&k_task<ACS_K_CONV, acs_args_conv>),
    reinterpret_cast<const void *>(&k_task<ACS_K_JOIN, acs_args_join>),
    reinterpret_cast<const void *>(&k_task<ACS_K_AVGPOOL, acs_args_avgpool>),
    reinterpret_cast<const void *>(&k_task<ACS_K_FC, acs_args_fc>),
    reinterpret_cast<const void *>(&k_task<ACS_K_COPY, acs_args_copy>),
    reinterpret_cast<const void *>(&k_task<ACS_K_SIGNAL, acs_args_signal>),
};
static_assert(sizeof(k_table) / sizeof(k_table[0]) == ACS_K_COUNT, "task table size");

const void *task_kernel(int32_t kid) { return (kid < 0 || kid >= ACS_K_COUNT) ? nullptr : k_table[kid]; }

hipError_t launch_task(int32_t kid, const void *args, uint32_t npieces, hipStream_t stream)
{
    if (kid < 0 || kid >= ACS_K_COUNT || k_table[kid] == nullptr || npieces == 0) return hipErrorInvalidValue;
    void *argv[2] = {const_cast<void *>(args), &npieces};
    return hipLaunchKernel(k_table[kid], dim3(npieces), dim3(ACS_BLOCK), argv, 0, stream);
}

// Several ready tasks of the plain path in one launch (they do not depend on
// each other): the task of a workgroup is found by a walk over the pieces,
// the same for every thread of it.
__global__ __launch_bounds__(ACS_BLOCK) void k_multi(MultiParams p)
{
    __shared__ __align__(16) uint8_t smem[kBodySmem];
    const uint32_t b = blockIdx.x;
    uint32_t i = 0;
    while (i + 1 < p.n && b >= p.t[i + 1].first) i++;
    run_body<false>(p.t[i].kid, p.t[i].args, b - p.t[i].first, p.t[i].np, smem);
}

hipError_t launch_multi(const MultiParams &p, hipStream_t stream)
{
    if (p.n == 0 || p.n > (uint32_t)kMultiMax || p.total == 0) return hipErrorInvalidValue;
    MultiParams copy = p;
    void *argv[1] = {&copy};
    return hipLaunchKernel(reinterpret_cast<const void *>(&k_multi), dim3(p.total), dim3(ACS_BLOCK), argv, 0, stream);
}

// One instance per bound on the window groups (1, 2, 4, 8), so that a
// single window does not carry the register pressure of eight.
template <int NG>
__global__ __launch_bounds__(ACS_BLOCK) void k_persistent(DevParams p)
{
    __shared__ __align__(16) uint8_t smem[kBodySmem];
    __shared__ Mail mail;
    if (blockIdx.x == 0) {
        FetchShared *fs = reinterpret_cast<FetchShared *>(smem);
        if (threadIdx.x == 0) fetch_init(fs);
        __syncthreads();
        const uint32_t wave = uni32(threadIdx.x) >> 6;   // uniform: whole waves take each branch
        if (wave == 0) window_wave<NG>(p, fs);
        else if (wave == 1) fifo_wave<NG>(p, fs);
        else if (NG == 1 && wave >= 2 && p.check_wave) check_wave(p, fs, wave - 2);
        return;
    }
    worker(p, smem, &mail);
}

// the smallest compiled group bound that covers the window's groups
static const void *persistent_kernel(int32_t n_groups)
{
    if (n_groups <= 1) return reinterpret_cast<const void *>(&k_persistent<1>);
    if (n_groups <= 2) return reinterpret_cast<const void *>(&k_persistent<2>);
    if (n_groups <= 4) return reinterpret_cast<const void *>(&k_persistent<4>);
    return reinterpret_cast<const void *>(&k_persistent<8>);
}

hipError_t launch_persistent(const DevParams &p, int32_t grid, hipStream_t stream)
{
    DevParams copy = p;
    void *argv[1] = {&copy};
    return hipLaunchKernel(persistent_kernel(p.n_groups), dim3(grid), dim3(ACS_BLOCK), argv, 0, stream);
}

hipError_t persistent_blocks_per_cu(int32_t n_groups, int32_t *blocks)
{
    int b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, persistent_kernel(n_groups), ACS_BLOCK, 0);
    *blocks = b;
    return e;
}

hipError_t persistent_lds_bytes(int32_t n_groups, int32_t *bytes)
{
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, persistent_kernel(n_groups));
    *bytes = (int32_t)a.sharedSizeBytes;
    return e;
}

}  // namespace acs
