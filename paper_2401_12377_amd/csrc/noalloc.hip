// Scheduler state of the windows configured without allocation
// (acs_window_configure_noalloc): one DevState per device in a static device
// array, and the fill kernel that clears it before each such window starts.
#include <hip/hip_runtime.h>

#include <mutex>

#include "acs_tasks.h"
#include "dev_shared.hpp"
#include "launch.hpp"

namespace acs {

static_assert(sizeof(DevState) % 256 == 0, "the state is cleared in 16-byte words and placed at 256 bytes");

// 1.6 MiB per device, placed when this code object is loaded on the device
// and held until the process ends.  In host code the array's name is a
// host-side stand-in: its device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address
// reaches kernels.
static __device__ __align__(256) DevState scratch[1];

constexpr int32_t kStaticDevices = 64;

hipError_t static_state(int32_t device, DevState **out)
{
    static std::mutex mu;
    static DevState *addr[kStaticDevices] = {};
    if (device < 0 || device >= kStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = static_cast<DevState *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

__global__ __launch_bounds__(ACS_BLOCK) void k_zero16(uint4 *p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * ACS_BLOCK + threadIdx.x; i < n; i += (uint64_t)gridDim.x * ACS_BLOCK)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t clear_state(DevState *st, hipStream_t stream)
{
    uint4 *p = reinterpret_cast<uint4 *>(st);
    uint64_t n = sizeof(DevState) / 16;
    void *argv[2] = {&p, &n};
    return hipLaunchKernel(reinterpret_cast<const void *>(&k_zero16), dim3(256), dim3(ACS_BLOCK), argv, 0, stream);
}

}  // namespace acs
