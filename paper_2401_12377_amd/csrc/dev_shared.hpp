// Structures shared by the host side of the device-resident path (built by
// the host compiler) and the persistent scheduler kernel (built by hipcc).
// Plain fixed-width fields only, so both compilers agree on the layout.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "acs.h"

namespace acs {

constexpr int kSegs = ACS_K_MAX;

// One submitted kernel as it travels from the host to the scheduler wave.
// Segments are stored as [start, end) with end saturated at 2^64 - 1; unused
// entries are the empty range [0, 0), which overlaps nothing.  The scheduler
// copies the first kDescCopyDwords words into the task table when it inserts
// the kernel (one 4-byte store per lane); the last 40 bytes hold what the
// scheduler fills in at dispatch for the workers and, in host-check mode,
// the upstream list the host computed.
struct DevDesc {
    uint64_t seq;
    int32_t kid;
    uint32_t npieces;
    uint32_t nseg;          // segments in use (reads and writes)
    uint32_t wbits;         // bit k set: segment k is a write
    uint64_t s[kSegs];
    uint64_t e[kSegs];
    uint8_t args[ACS_ARGS_MAX];
    // scheduler-owned part (the host leaves it zero)
    uint64_t wait_mask;     // window slots still running when the kernel was dispatched
    uint32_t ptarget;       // cnt[slot] after this kernel's last piece (npieces > 1; 64 per piece)
    uint32_t pad0;
    // host-check mode: bit d set when the host found the kernel submitted
    // d + 1 places earlier in conflict with this one (read by the window wave
    // from the staged copy; not part of the task table)
    uint64_t host_up;
    uint32_t pad[4];
};
static_assert(sizeof(DevDesc) == 256, "descriptor must be 256 bytes");
static_assert(offsetof(DevDesc, host_up) == 232, "host_up is dwords 58 and 59 of the descriptor");
constexpr uint32_t kDescCopyDwords = 54;   // dwords of DevDesc the task table needs
constexpr int kHostUpDword = 58;
constexpr int kSegStartDword = 6;          // s[k] is dwords 6 + 2k and 7 + 2k
constexpr int kSegEndDword = 22;           // e[k] is dwords 22 + 2k and 23 + 2k
static_assert(offsetof(DevDesc, s) == 4 * kSegStartDword && offsetof(DevDesc, e) == 4 * kSegEndDword,
              "segment dwords");

constexpr int kMaxGroups = 8;   // independent windows served by one window wave

// Host-resident control block (pinned, coherent).  The first 128 bytes are
// written by the host (one tail per window group, then stop and the snapshot
// request), the rest by the device.
struct HostCtrl {
    volatile uint64_t tail[kMaxGroups];     // descriptors published by the host, per group
    volatile uint64_t stop;                 // 1: exit when idle, 2: abort now
    volatile uint64_t snap_req;             // bumped by the host to ask for a window snapshot
    uint64_t pad0[6];
    volatile uint64_t consumed[kMaxGroups]; // descriptors copied off each group's ring by the device
    volatile uint64_t retired[kMaxGroups];  // kernels completed, per group
    volatile uint64_t error;                // sticky device-side error code (0 = none)
    volatile uint64_t snap_ack;             // last snapshot request served
    volatile uint64_t snap_count;           // entries in the snapshot
    volatile uint64_t alive;                // set when the scheduler wave starts
    volatile uint64_t exited;               // set when the scheduler wave leaves
    volatile uint64_t checks;               // overlap tests made by the window wave (statistics)
    volatile uint64_t check_wave_tests[2];  // overlap tests made by each check wave (statistics)
    volatile uint64_t published;            // work-queue entries published, sentinels excluded (at exit)
    acs_entry snap[ACS_W_MAX];
};

// The task table holds, per window slot, the descriptor of the kernel in
// that slot.  A kernel is handed to the workers as soon as every kernel it
// waits for has been handed out; wait_mask and wait_target then tell its
// workers which completion words must reach which values before the body may
// start.
//
// Completion is signalled with a device-scope store: the worker that
// finishes a kernel's last piece writes seq + 1 (mod 2^32) into done[slot].
// A store reaches another XCD's polling load in a few hundred nanoseconds,
// an atomic read-modify-write takes several times longer, so the per-slot
// piece counter cnt[] is touched only by kernels of more than one piece, to
// find which piece is the last.
using TaskEntry = DevDesc;

constexpr uint32_t kQueueCap = 1u << 16;       // work queue entries (power of two)
constexpr uint32_t kMaxPieces = 256;           // pieces per task
constexpr uint32_t kSentinelSlot = 0xFF;

// Device-resident scheduler state (device memory).
struct DevState {
    uint64_t deq;                 // work-queue tickets taken by workers, 64 per ticket
    uint64_t pad0[31];
    uint32_t cnt[ACS_W_MAX];      // per-slot piece counters, 64 per piece (monotonic, multi-piece kernels only)
    uint64_t pad1[32];
    uint32_t done[ACS_W_MAX];     // per-slot completion words: seq + 1 of the last kernel finished
    uint64_t pad2[32];
    TaskEntry task[ACS_W_MAX];
    uint32_t wait_target[ACS_W_MAX][ACS_W_MAX];   // [slot][upstream slot]: done[] value to wait for
    uint64_t ent[kQueueCap];      // work-queue entries: tag(32) | slot(8) | piece(24)
};

struct DevParams {
    HostCtrl *ctrl;
    DevDesc *ring;                // host-resident descriptor rings, group g at ring + g * (ring_mask + 1)
    DevState *st;
    acs_trace_rec *trace;         // device trace (or null), indexed by sequence number
    uint32_t ring_mask;
    uint32_t trace_cap;
    int32_t W;                    // slots per group
    int32_t n_workers;
    int32_t n_groups;             // independent windows, 1..kMaxGroups; n_groups * pow2(W) <= 64
    int32_t host_check;           // 0: dependency checks in the window wave; M > 0: each kernel comes
                                  // checked against the M submitted before it (one window only)
    int32_t check_wave;           // 1: a wave ahead of the window makes those checks (M = 64); 0: the host
};

}  // namespace acs
