// Structures shared by the host side of the device-resident path (built by
// the host compiler) and the persistent scheduler kernel (built by hipcc).
// Plain fixed-width fields only, so both compilers agree on the layout.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "acs.h"

namespace acs {

constexpr int kSegs = ACS_K_MAX;

// One submitted kernel as it travels from the host to the scheduler.
// Segments are stored as [start, end) with end saturated at 2^64 - 1; unused
// entries are the empty range [0, 0), which overlaps nothing.  gseq numbers
// the kernels of one window group without gaps (0, 1, 2, ...); completions
// and dependency distances are kept in that numbering.  The FIFO wave copies
// every descriptor, as the host wrote it, into the device-memory ring the
// workers read (DevState::dring, at its group and gseq), and stages it in
// LDS for the window.  Everything the window and the workers need when the
// host makes the dependency checks sits in the first 128 bytes, the ranges
// (needed only by checks on the device) in the last 128: in host-check mode
// only the first half crosses from host memory.
struct DevDesc {
    uint64_t seq;           // submission index over all groups (traces)
    int32_t kid;
    uint32_t npieces;
    uint32_t gseq;          // index of the kernel within its window group
    uint32_t group;
    // bit b set: the kernel of the same group with gseq - 1 - b conflicts
    // with this one.  Written by the host (host-check mode), by a check wave
    // into the staged copy (the window then writes it into the ring), or by
    // the window wave after its own checks.
    uint64_t host_up;
    uint8_t args[ACS_ARGS_MAX];
    uint32_t nseg;          // segments in use (reads and writes)
    uint32_t wbits;         // bit k set: segment k is a write
    // bit b set: the kernel with gseq - 65 - b conflicts (host checks
    // against more than 64 kernels only; zero otherwise)
    uint64_t host_up_hi;
    uint32_t pad[4];
    uint64_t s[kSegs];
    uint64_t e[kSegs];
};
static_assert(sizeof(DevDesc) == 256, "descriptor must be 256 bytes");
constexpr int kKidDword = 2;
constexpr int kNpiecesDword = 3;
constexpr int kGseqDword = 4;
constexpr int kHostUpDword = 6;
constexpr int kNsegDword = 24;
constexpr int kWbitsDword = 25;
constexpr int kHostUpHiDword = 26;
constexpr int kSegStartDword = 32;         // s[k] is dwords 32 + 2k and 33 + 2k
constexpr int kSegEndDword = 48;           // e[k] is dwords 48 + 2k and 49 + 2k
constexpr uint32_t kDescHeadBytes = 128;   // what the window and workers read
static_assert(offsetof(DevDesc, kid) == 4 * kKidDword && offsetof(DevDesc, npieces) == 4 * kNpiecesDword &&
                  offsetof(DevDesc, gseq) == 4 * kGseqDword && offsetof(DevDesc, host_up) == 4 * kHostUpDword &&
                  offsetof(DevDesc, nseg) == 4 * kNsegDword && offsetof(DevDesc, wbits) == 4 * kWbitsDword &&
                  offsetof(DevDesc, host_up_hi) == 4 * kHostUpHiDword,
              "descriptor dwords");
static_assert(offsetof(DevDesc, s) == 4 * kSegStartDword && offsetof(DevDesc, e) == 4 * kSegEndDword,
              "segment dwords");
static_assert(offsetof(DevDesc, args) + ACS_ARGS_MAX <= kDescHeadBytes && offsetof(DevDesc, s) == kDescHeadBytes,
              "the head holds everything but the ranges");

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

// Completion.  The worker that finishes a kernel's last piece stores gseq + 1
// into dseq[group][gseq % kSeqRing] (a device-scope store: it reaches a
// polling wave on another XCD in a few hundred nanoseconds, an atomic
// read-modify-write takes several times longer).  The window wave polls the
// word of each kernel it holds; a worker whose kernel depends on kernel k of
// its group waits until dseq[group][k % kSeqRing] has reached k + 1.  The
// ring is large enough because no two kernels of one group in flight (or
// waited for) are kSeqRing apart: admission holds a kernel while one 64 or
// more older is still in the window (up to ACS_HOST_CHECK_MAX with the
// checks on the host), and dependencies reach back no further.
// Kernels of several pieces count their pieces in cnt[group][gseq %
// kSeqRing] first (64 per piece); the last piece resets the counter before
// it marks the kernel complete.
//
// Work queue entries: tag (8 bits: (ticket >> 16) + 1, so that an entry left
// from an earlier lap of the queue never matches) | group (8; kSentinelGroup
// tells a worker to leave) | piece (16) | gseq (32).
constexpr uint32_t kQueueCap = 1u << 16;       // work queue entries (power of two)
constexpr uint32_t kMaxPieces = 256;           // pieces per task
constexpr uint32_t kSentinelGroup = 0xFF;
constexpr uint32_t kSeqRing = 512;             // completion words per group
constexpr uint32_t kDescRing = 512;            // device descriptor ring entries per group

constexpr uint64_t queue_entry(uint64_t ticket, uint32_t group, uint32_t piece, uint32_t gseq)
{
    return ((((ticket >> 16) + 1) & 0xFFull) << 56) | ((uint64_t)(group & 0xFFu) << 48) |
           ((uint64_t)(piece & 0xFFFFu) << 32) | gseq;
}

// Device-resident scheduler state (device memory).
struct DevState {
    uint64_t deq;                 // work-queue tickets taken by workers, 64 per ticket
    uint64_t pad0[31];
    uint32_t dseq[kMaxGroups][kSeqRing];
    uint32_t cnt[kMaxGroups][kSeqRing];
    DevDesc dring[kMaxGroups][kDescRing];
    uint64_t ent[kQueueCap];
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
