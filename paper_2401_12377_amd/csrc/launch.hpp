// Host-callable entry points of the HIP translation unit (kernels.hip).
#pragma once
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "acs.h"
#include "dev_shared.hpp"

namespace acs {

// Launches the standalone kernel of task `kid` with `npieces` workgroups of
// 256 threads on `stream`.  `args` points at the task's argument struct.
hipError_t launch_task(int32_t kid, const void *args, uint32_t npieces, hipStream_t stream);

// The standalone kernel of task `kid` (for graph nodes), or null.
const void *task_kernel(int32_t kid);

// Several mutually independent tasks in one launch: workgroup b runs piece
// b - first of the task whose pieces [first, first + np) hold b.
constexpr int32_t kMultiMax = 32;
struct MultiTask {
    int32_t kid;
    uint32_t np;
    uint32_t first;
    uint32_t pad;
    uint8_t args[ACS_ARGS_MAX];
};
struct MultiParams {
    uint32_t n;        // tasks
    uint32_t total;    // workgroups: the sum of the tasks' pieces
    MultiTask t[kMultiMax];
};
hipError_t launch_multi(const MultiParams &p, hipStream_t stream);

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
