// Host-callable entry points of the HIP translation unit (kernels.hip).
#pragma once
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "dev_shared.hpp"

namespace acs {

// Launches the standalone kernel of task `kid` with `npieces` workgroups of
// 256 threads on `stream`.  `args` points at the task's argument struct.
hipError_t launch_task(int32_t kid, const void *args, uint32_t npieces, hipStream_t stream);

// The standalone kernel of task `kid` (for graph nodes), or null.
const void *task_kernel(int32_t kid);

// Launches the persistent scheduler kernel: workgroup 0 holds the window,
// workgroups 1 .. grid-1 are workers.
hipError_t launch_persistent(const DevParams &p, int32_t grid, hipStream_t stream);

// Workgroups of the persistent kernel (the instance for n_groups window
// groups) that fit on one compute unit.
hipError_t persistent_blocks_per_cu(int32_t n_groups, int32_t *blocks);

// Static LDS of one persistent-kernel workgroup (instance for n_groups).
hipError_t persistent_lds_bytes(int32_t n_groups, int32_t *bytes);

// Device address of this device's static scheduler state (the state of the
// windows configured without allocation), taken with the device current.
hipError_t static_state(int32_t device, DevState **out);

// Zeroes a scheduler state with a fill kernel on `stream`.
hipError_t clear_state(DevState *st, hipStream_t stream);

}  // namespace acs
