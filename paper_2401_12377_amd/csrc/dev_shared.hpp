// Structures shared by the host side of the device-resident path (built by
// the host compiler) and the persistent scheduler kernel (built by hipcc).
// Plain fixed-width fields only, so both compilers agree on the layout.
#pragma once
#include <stdint.h>

#include "acs.h"

namespace acs {

constexpr int kSegs = ACS_K_MAX;

// One submitted kernel as it travels from the host to the scheduler wave.
// Segments are stored as [start, end) with end saturated at 2^64 - 1; unused
// entries are the empty range [0, 0), which overlaps nothing.
struct DevDesc {
    uint64_t seq;
    int32_t kid;
    uint32_t npieces;
    uint32_t nseg;          // segments in use (reads and writes)
    uint32_t wbits;         // bit k set: segment k is a write
    uint64_t s[kSegs];
    uint64_t e[kSegs];
    uint8_t args[ACS_ARGS_MAX];
    uint8_t pad[40];
};
static_assert(sizeof(DevDesc) == 256, "descriptor must be 256 bytes");

// Host-resident control block (pinned, coherent).  The first cache line is
// written by the host, the rest by the device.
struct HostCtrl {
    volatile uint64_t tail;       // descriptors published by the host
    volatile uint64_t stop;       // 1: exit when idle, 2: abort now
    volatile uint64_t snap_req;   // bumped by the host to ask for a window snapshot
    uint64_t pad0[13];
    volatile uint64_t consumed;   // descriptors copied off the ring by the device
    volatile uint64_t retired;    // kernels completed
    volatile uint64_t error;      // sticky device-side error code (0 = none)
    volatile uint64_t snap_ack;   // last snapshot request served
    volatile uint64_t snap_count; // entries in the snapshot
    volatile uint64_t alive;      // set when the scheduler wave starts
    volatile uint64_t exited;     // set when the scheduler wave leaves
    volatile uint64_t checks;     // overlap tests made (statistics)
    uint64_t pad1[8];
    acs_entry snap[ACS_W_MAX];
};

// What a worker needs to run one piece of a task: copied by the scheduler
// into the slot's entry of the task table when the kernel is inserted.
// A kernel is handed to the workers as soon as every kernel it waits for has
// been handed out; wait_mask / wait_target then tell its workers which
// completion counters must reach which values before the body may start.
struct TaskEntry {
    int32_t kid;
    uint32_t npieces;
    uint64_t seq;
    uint8_t args[ACS_ARGS_MAX];
    uint64_t wait_mask;                   // window slots still running when dispatched
    uint32_t pad0[2];
    uint32_t wait_target[ACS_W_MAX];      // completion-counter value that means "done"
    uint8_t pad[160];
};
static_assert(sizeof(TaskEntry) == 512, "task entry must be 512 bytes");

constexpr uint32_t kQueueCap = 1u << 16;       // work queue entries (power of two)
constexpr uint32_t kMaxPieces = 256;           // pieces per task
constexpr uint32_t kSentinelSlot = 0xFF;

// Device-resident scheduler state (device memory).
struct DevState {
    uint64_t deq;                 // work-queue tickets taken by workers
    uint64_t pad0[31];
    uint32_t cnt[ACS_W_MAX];      // per-slot completion counters (monotonic)
    uint64_t pad1[32];
    TaskEntry task[ACS_W_MAX];
    uint64_t ent[kQueueCap];      // work-queue entries: tag(32) | slot(8) | piece(24)
};

struct DevParams {
    HostCtrl *ctrl;
    DevDesc *ring;                // host-resident descriptor ring
    DevState *st;
    acs_trace_rec *trace;         // device trace (or null)
    uint32_t ring_mask;
    uint32_t trace_cap;
    int32_t W;
    int32_t n_workers;
};

}  // namespace acs
