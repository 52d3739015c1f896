// Wave-level building blocks of the persistent scheduler kernel (device code).
//
// Workgroup 0 is the window:
//   wave 0  the window module.  Lane i owns window slot i: the group
//           sequence number, piece count and upstream list (by distance) of
//           the kernel it holds live in that lane's registers.  A pass admits
//           every staged kernel that finds a free slot, in submission order,
//           and publishes it to the workers at once: a kernel may start as
//           soon as it is handed out, because its workers wait for the
//           completion words of its upstream kernels themselves.  Completions
//           are seen by polling those words; a ballot of the finished slots
//           frees them.  With one window and the checks made ahead of it
//           (check waves or the host) a pass handles all its kernels in
//           lane-parallel steps; otherwise the wave tests each new kernel's
//           ranges against its slots (Algorithm 1, both directions), one
//           kernel per group per step, and turns the ballot of conflicting
//           slots into the same upstream list.
//   wave 1  the input FIFO: copies descriptors from the host-resident rings
//           into the device-memory ring the workers read and into small
//           rings in LDS for the window, so that host-memory latency never
//           stalls the window loop.
//   waves 2 and 3  (one window, checks ahead of the window) test each staged
//           kernel against the 64 submitted before it, alternating between
//           them, then hand it on to the window wave.
// The lanes of the window wave may be split into up to eight groups, each an
// independent window with its own input ring (for many independent task
// graphs in one launch).
// Workgroups 1.. are workers: each takes a ticket from the work queue, waits
// for the entry with that ticket, reads the kernel's descriptor, waits until
// the kernels it depends on have completed, runs one piece of the task body
// and, for the last piece, stores the kernel's completion word.
//
// Visibility between the waves runs on device-scope stores.  Every store that
// another workgroup reads (descriptors, task results, completion words) is a
// device-scope store, which the hardware writes through the L2 of the storing
// XCD (the XCDs' L2 caches are not coherent with each other), and it is
// complete once the storing wave's vector-memory counter has drained.  So a
// wave publishes by waiting for its own stores and then storing the word
// that announces them; the reader acquires (invalidating its stale cache
// lines) after it has seen that word.  A release at device scope would
// instead write back the whole L2 of the XCD, which serialises the pieces of
// a wide kernel.
//
// Only HIP device built-ins are used here, so the same source also builds
// for the host against an emulation of those built-ins (a CPU build used by
// the tests to run the scheduler logic without a GPU).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bodies.hpp"
#include "dev_shared.hpp"

namespace acs {

constexpr uint32_t kWave = 64;        // lanes of a wavefront
constexpr uint32_t kLdsDescs = 128;   // descriptors staged in LDS (32 KB), shared by the groups (lds_depth)
constexpr uint32_t kAdmitBatch = 16;  // kernels per group admitted per loop with checks at insert
constexpr uint32_t kSpan = 64;        // a kernel waits while one kSpan or more older (same
                                      // group) is in the window: upstream lists reach back 64
constexpr uint32_t kHostSpan = ACS_HOST_CHECK_MAX;   // the same with the checks on the host
static_assert(kHostSpan >= kSpan && kHostSpan <= 128, "upstream lists are two 64-bit words");
// Kernels in flight span at most kHostSpan + 1 sequence numbers and wait for
// kernels at most kHostSpan before them: no two live completion words share a
// place in the ring.
static_assert(kSeqRing >= 2 * kHostSpan + 2, "completion ring must cover two spans");
static_assert(kDescRing >= kLdsDescs + 2 * kHostSpan + 1, "descriptor ring must cover staging and window");

struct FetchShared {
    uint32_t tail[kMaxGroups];   // descriptors ready for the window wave per group (FIFO or check wave)
    uint32_t staged;             // checks ahead of the window: descriptors copied, not yet checked
    uint32_t recorded[2];        // checks ahead of the window: descriptors each check wave has read
    uint32_t head[kMaxGroups];   // descriptors taken per group (written by the window wave)
    uint32_t stop;               // mirror of the host stop flag
    uint32_t exit;               // window wave -> FIFO wave: leave
    uint64_t snap_req;           // mirror of the host snapshot request counter
    DevDesc ring[kLdsDescs];     // group g: ring[g * depth, (g + 1) * depth)
};
static_assert(sizeof(FetchShared) <= kBodySmem, "FIFO staging must fit the LDS scratch");

// Staging slots per group: a power of two (the share of kLdsDescs for the
// group count rounded up to a power of two), so positions are a mask.
__device__ inline uint32_t lds_depth(int32_t groups)
{
    return groups <= 1 ? kLdsDescs : kLdsDescs >> (32u - (uint32_t)__builtin_clz((uint32_t)groups - 1u));
}

// by one thread of workgroup 0, before the workgroup barrier that starts the waves
__device__ inline void fetch_init(FetchShared *fs)
{
    for (int g = 0; g < kMaxGroups; g++) fs->tail[g] = fs->head[g] = 0;
    fs->staged = 0;
    fs->recorded[0] = fs->recorded[1] = 0;
    fs->stop = 0;
    fs->exit = 0;
    fs->snap_req = 0;
}

struct Mail {
    uint32_t group, piece;
    int32_t kid;
    uint32_t np, gseq, pad;
    uint64_t seq;
    uint64_t t0;
    uint8_t args[ACS_ARGS_MAX];
};

#define LDS_LOAD(p) __hip_atomic_load((p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
#define LDS_STORE(p, v) __hip_atomic_store((p), (v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)

// A value every lane of the wave must agree on is taken from the first lane,
// so control flow that depends on it is uniform by construction.
__device__ inline uint32_t uni32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ inline uint64_t uni64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// readlane returns int: every use goes through these, which zero-extend
__device__ inline uint32_t readlane32(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }
__device__ inline uint64_t readlane64(uint64_t x, int l)
{
    const uint32_t lo = readlane32((uint32_t)x, l);
    const uint32_t hi = readlane32((uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
// a 64-bit field held in dwords l (low) and l + 1 (high) of a wave-wide word
__device__ inline uint64_t readpair(uint32_t x, int l) { return ((uint64_t)readlane32(x, l + 1) << 32) | readlane32(x, l); }

// The dependency checks of a single window made while kernels are staged
// (the host/device split of Section IV-C with the host's part done by the
// FIFO wave): every kernel is tested, in submission order, against the 64
// submitted before it.  Lane l keeps the ranges of the latest kernel whose
// group sequence number is l mod 64, so one pass tests all 64 at once (Algorithm 1
// in both directions, as in the window wave).  A new read can only meet a
// write, so it is tested against the first two positions only while no
// kernel so far had a write at a later position (mw); the library lists a
// kernel's writes before its reads, which keeps mw at the most writes any
// kernel has.
// The result goes into the staged descriptor as the upstream-by-distance
// word of host-check mode: bit b set when the kernel submitted b + 1 places
// earlier conflicts.  The window wave keeps from it the kernels still in the
// window.
struct SeqHistory {
    uint64_t s[kSegs], e[kSegs];   // ranges of this lane's kernel; unused: empty [0, 0)
    uint32_t w;                    // bit m: position m is a write
    uint32_t mw;                   // highest write position + 1 of any kernel so far (the same on
                                   // every lane)
    uint32_t mn;                   // most positions any kernel so far uses (the same on every lane)
};

__device__ inline void history_init(SeqHistory &h)
{
#pragma unroll
    for (int m = 0; m < kSegs; m++) h.s[m] = h.e[m] = 0;
    h.w = 0;
    h.mw = 0;
    h.mn = 0;
}

// d: the staged descriptor (LDS).  test: check the kernel and write its
// upstream word (else only record it); returns the pair tests made.
__device__ inline uint64_t history_check(DevDesc *d, SeqHistory &h, uint32_t lane, bool test)
{
    const uint32_t dw = reinterpret_cast<const uint32_t *>(d)[lane];
    // the new kernel's ranges, for its place in the history: loaded by every
    // lane (one address, a broadcast) now, so that the wait overlaps the tests
    uint64_t ns[kSegs], ne[kSegs];
#pragma unroll
    for (int m = 0; m < kSegs; m++) {
        ns[m] = d->s[m];
        ne[m] = d->e[m];
    }
    const uint32_t gq = readlane32(dw, kGseqDword);
    const uint32_t nraw = readlane32(dw, kNsegDword);
    const uint32_t nseg = nraw < (uint32_t)kSegs ? nraw : (uint32_t)kSegs;
    const uint32_t segmask = (1u << nseg) - 1u;
    const uint32_t wb = readlane32(dw, kWbitsDword) & segmask;
    const uint32_t wtop = wb ? 32u - (uint32_t)__builtin_clz(wb) : 0u;
    // The new ranges are the broadcast values above (no readlane per range);
    // positions beyond any kernel's count so far hold [0, 0) everywhere and
    // are skipped.  Every branch here is on wave-uniform values.
    const uint32_t mn = h.mn > nseg ? h.mn : nseg;
    bool hit = false;
#pragma unroll
    for (int k = 0; k < kSegs; k++) {
        if (!test || (uint32_t)k >= nseg) break;
        const uint64_t a0 = ns[k], a1 = ne[k];
        if ((wb >> k) & 1u) {
            // a new write meets any intersecting range
#pragma unroll
            for (int m = 0; m < kSegs; m++)
                if ((uint32_t)m < mn) hit |= a0 < h.e[m] && a1 > h.s[m];
        } else {
            // a new read meets only writes, which sit at the first mw positions
#pragma unroll
            for (int m = 0; m < kSegs; m++)
                if ((uint32_t)m < h.mw) hit |= a0 < h.e[m] && a1 > h.s[m] && ((h.w >> m) & 1u);
        }
    }
    const uint32_t nw = (uint32_t)__builtin_popcount(wb);
    const uint64_t tests =
        test ? (uint64_t)(nw * mn + (nseg - nw) * h.mw) * (gq < 64u ? gq : 64u) : 0ull;
    // bit b of the result is the kernel b + 1 places back, held by lane
    // r - b mod 64 (r = gq - 1 mod 64): the lane mask reversed (lane l to
    // bit 63 - l) and rotated right by 63 - r.  There is none when b >= gq.
    const uint64_t hm = __builtin_amdgcn_ballot_w64(hit);
    const uint32_t rot = (63u - ((gq - 1u) & 63u)) & 63u;
    const uint64_t rv = __builtin_bitreverse64(hm);
    uint64_t up = rot ? ((rv >> rot) | (rv << (64u - rot))) : rv;
    if (gq < 64u) up &= (1ull << gq) - 1ull;
    uint32_t *words = reinterpret_cast<uint32_t *>(d);
    if (test && lane == 0) {
        words[kHostUpDword] = (uint32_t)up;
        words[kHostUpDword + 1] = (uint32_t)(up >> 32);
    }
    // the kernel takes its place in the history
    if (lane == (gq & 63u)) {
#pragma unroll
        for (int m = 0; m < kSegs; m++) {
            h.s[m] = (uint32_t)m < nseg ? ns[m] : 0ull;
            h.e[m] = (uint32_t)m < nseg ? ne[m] : 0ull;
        }
        h.w = wb;
    }
    h.mw = wtop > h.mw ? wtop : h.mw;
    h.mn = mn;
    return tests;
}

// NG: compile-time bound on the group count (1, 2, 4 or 8), so that the
// per-group loops disappear for a single window
template <int NG>
__device__ inline void fifo_wave(const DevParams &p, FetchShared *fs)
{
    const uint32_t lane = threadIdx.x & 63u;
    const int32_t G = p.n_groups;
    ACS_GAS HostCtrl *const ctrl = gp(p.ctrl);
    ACS_GAS DevState *const st = gp(p.st);
    // one window: a constant, so that ring positions are a mask, not a division
    const uint32_t depth = NG == 1 ? kLdsDescs : lds_depth(G), ring_cap = p.ring_mask + 1;
    // With the checks on the host only each descriptor's first half is
    // copied (8 chunks of 16 bytes instead of 16): 8 descriptors per row of
    // the wave instead of 4.
    const bool half = NG == 1 && p.host_check > 0 && p.check_wave == 0;
    const uint32_t lgc = half ? 3u : 4u;           // log2 of the 16-byte chunks copied per descriptor
    constexpr uint32_t kRows = 8;
    const uint32_t jobs = kRows << (6u - lgc);     // descriptors per copy round
    uint64_t consumed[NG], htail[NG], told[NG];
    uint32_t ftail[NG];
#pragma unroll
    for (int g = 0; g < NG; g++) consumed[g] = htail[g] = told[g] = ftail[g] = 0;
    // The host needs `consumed` only for back-pressure on its ring, so it is
    // published every ring_cap / 8 descriptors and when the wave goes idle:
    // a store to host memory per copy would make every copy wait for it.
    const uint64_t tell_every = ring_cap / 8 > 0 ? ring_cap / 8 : 1;
    // checks ahead of the window: the copies go to the check wave instead
    const bool fc = NG == 1 && p.check_wave != 0;
    for (;;) {
        if (uni32(LDS_LOAD(&fs->exit))) break;
        // Each round issues, together: the loads of the host's control lines
        // (the tails, stop and the snapshot request) and the loads of up to
        // 32 descriptors that earlier rounds already know to be published.
        // So one round costs one round trip to host memory.
        uint64_t t[NG];
#pragma unroll
        for (int g = 0; g < NG; g++)
            t[g] = g < G ? __hip_atomic_load(&ctrl->tail[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0ull;
        const uint64_t s0 = __hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint64_t sr = __hip_atomic_load(&ctrl->snap_req, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        // Job j of the round is descriptor consumed[g] + (j - start[g]) of the
        // group g whose range [start[g], start[g] + cnt[g]) holds j.
        uint32_t cnt[NG], start[NG], total = 0;
#pragma unroll
        for (int g = 0; g < NG; g++) {
            cnt[g] = 0;
            start[g] = total;
            if (g < G) {
                // a slot is free once the window wave took its kernel and, with
                // the checks ahead of the window, both check waves read it
                uint32_t freed = uni32(LDS_LOAD(&fs->head[g]));
                if (fc) {
                    const uint32_t r0 = uni32(LDS_LOAD(&fs->recorded[0])), r1 = uni32(LDS_LOAD(&fs->recorded[1]));
                    freed = (int32_t)(r0 - freed) < 0 ? r0 : freed;
                    freed = (int32_t)(r1 - freed) < 0 ? r1 : freed;
                }
                const uint32_t space = depth - (ftail[g] - freed);
                const uint64_t avail = htail[g] - consumed[g];
                uint32_t n = avail < space ? (uint32_t)avail : space;
                if (n > jobs - total) n = jobs - total;
                cnt[g] = n;
                total += n;
            }
        }
        // 16 bytes per lane per row: lane l of row r copies chunk l % c of
        // job (64 / c) r + l / c, c = the chunks copied per descriptor
        uint4 v[kRows];
        uint32_t dst_off[kRows];
        ACS_GAS uint64_t *ddst[kRows];   // the chunk's place in the device descriptor ring
#pragma unroll
        for (int r = 0; r < (int)kRows; r++) {
            const uint32_t j = ((uint32_t)r << (6u - lgc)) + (lane >> lgc), c = lane & ((1u << lgc) - 1u);
            uint32_t gg = 0, ii = 0, ft = 0;
            uint64_t cons = 0;
#pragma unroll
            for (int g = 0; g < NG; g++)
                if (j >= start[g] && j < start[g] + cnt[g]) {
                    gg = (uint32_t)g;
                    ii = j - start[g];
                    cons = consumed[g];
                    ft = ftail[g];
                }
            // Every lane loads, the lanes without a job from the ring's first
            // slot (always mapped; the value is dropped): a load under a
            // branch gets its own wait for completion, and the rows' host
            // reads would follow each other instead of overlapping.
            const bool job = j < total;
            const ACS_GAS DevDesc *src =
                gp(p.ring) + (job ? (uint64_t)gg * ring_cap + ((cons + ii) & p.ring_mask) : 0ull);
            v[r] = ld4(reinterpret_cast<const ACS_GAS uint4 *>(src) + c);
            dst_off[r] = job ? (gg * depth + ((ft + ii) & (depth - 1u))) * 256u + c * 16u : ~0u;
            // the descriptor's group sequence number is its place in the group's ring
            ddst[r] = job ? reinterpret_cast<ACS_GAS uint64_t *>(&st->dring[gg][(uint32_t)(cons + ii) & (kDescRing - 1u)]) +
                                2u * c
                          : nullptr;
        }
        // control lines: newly published descriptors are read in later
        // rounds, after this acquire
        bool fresh = false;
#pragma unroll
        for (int g = 0; g < NG; g++) {
            const uint64_t nt = uni64(t[g]);
            fresh |= nt != htail[g];
            htail[g] = nt;
        }
        const uint64_t st = uni64(s0);
        const uint64_t sru = uni64(sr);
        if (lane == 0) {
            LDS_STORE(&fs->stop, (uint32_t)st);
            LDS_STORE(&fs->snap_req, sru);
        }
        if (fresh) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        if (total > 0) {
            // the copy the workers read, with device scope (they run on
            // other XCDs); complete before the window can hand the kernel out
#pragma unroll
            for (int r = 0; r < (int)kRows; r++)
                if (ddst[r]) {
                    __hip_atomic_store(ddst[r], ((uint64_t)v[r].y << 32) | v[r].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(ddst[r] + 1, ((uint64_t)v[r].w << 32) | v[r].z, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
            for (int r = 0; r < (int)kRows; r++)
                if (dst_off[r] != ~0u) *reinterpret_cast<uint4 *>(reinterpret_cast<char *>(fs->ring) + dst_off[r]) = v[r];
            // 0x0F70: vmcnt 0, expcnt 7, lgkmcnt 15
            __builtin_amdgcn_s_waitcnt(0x0F70);
            // every lane's part of the copy lands before lane 0 publishes it
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
#pragma unroll
            for (int g = 0; g < NG; g++) {
                if (cnt[g] == 0) continue;
                ftail[g] += cnt[g];
                consumed[g] += cnt[g];
                if (lane == 0) LDS_STORE(fc ? &fs->staged : &fs->tail[g], ftail[g]);
                if (consumed[g] - told[g] >= tell_every) {
                    if (lane == 0)
                        __hip_atomic_store(&ctrl->consumed[g], consumed[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    told[g] = consumed[g];
                }
            }
        } else {
#pragma unroll
            for (int g = 0; g < NG; g++)
                if (g < G && told[g] != consumed[g]) {
                    if (lane == 0)
                        __hip_atomic_store(&ctrl->consumed[g], consumed[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    told[g] = consumed[g];
                }
            if (st == 2) break;   // host abort: leave even if the window wave is gone
            if (!fresh) __builtin_amdgcn_s_sleep(1);
        }
    }
}

// Waves 2 and 3 when the checks run ahead of the window (one window): both
// take every kernel the FIFO wave staged, in order, and record it in their
// own copy of the history; wave 2 + c checks the kernels of staged index
// c mod 2 and hands each to the window wave once the other wave has handed
// on the kernel before it, so kernels reach the window in order while two
// checks run at once.  They leave with the window wave, or on an abort.
__device__ inline void check_wave(const DevParams &p, FetchShared *fs, uint32_t c)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t depth = lds_depth(1);
    SeqHistory hist;
    history_init(hist);
    uint64_t tests = 0;
    uint32_t done = 0;
    bool abort = false;
    while (!abort) {
        const uint32_t staged = uni32(LDS_LOAD(&fs->staged));
        if (staged == done) {
            if (uni32(LDS_LOAD(&fs->exit)) || uni32(LDS_LOAD(&fs->stop)) == 2u) break;
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (; done != staged; done++) {
            const bool mine = (done & 1u) == c;
            tests += history_check(&fs->ring[done & (depth - 1u)], hist, lane, mine);
            // this wave is done reading the staged descriptor
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) LDS_STORE(&fs->recorded[c], done + 1);
            if (!mine) continue;
            // the kernel before this one is handed on by the other wave
            for (uint32_t spin = 1; uni32(LDS_LOAD(&fs->tail[0])) != done; spin++) {
                if ((spin & 255u) == 0 && uni32(LDS_LOAD(&fs->stop)) == 2u) {
                    abort = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (abort) break;
            // the upstream word lands before the kernel is handed on
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) LDS_STORE(&fs->tail[0], done + 1);
        }
    }
    if (lane == 0)
        __hip_atomic_store(&gp(p.ctrl)->check_wave_tests[c], tests, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Trace records are written with device-scope stores like everything else
// that workers touch: workers update t_start and t_end of a record with
// atomics, which the write-back of a plain store's dirty bytes from the
// window wave's L2 could later overwrite.
__device__ inline void tput(ACS_GAS int64_t *f, int64_t v) { __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ inline void trace_insert(ACS_GAS acs_trace_rec *r, uint64_t seq, int32_t slot, int32_t kid, uint64_t ev, uint64_t valid,
                                    uint64_t up)
{
    tput(&r->seq, (int64_t)seq);
    tput(&r->slot, slot);
    tput(&r->kernel_id, kid);
    tput(&r->ev_insert, (int64_t)ev);
    tput(&r->ev_dispatch, -1);
    tput(&r->ev_retire, -1);
    tput(reinterpret_cast<ACS_GAS int64_t *>(&r->valid_mask), (int64_t)valid);
    tput(reinterpret_cast<ACS_GAS int64_t *>(&r->up_mask), (int64_t)up);
    tput(&r->t_start, INT64_MAX);
    tput(&r->t_end, 0);
    tput(&r->t_dispatch, -1);
    tput(&r->t_retire, -1);
}

// Pair tests of one insertion pass (Algorithm 1 in both directions): segment
// k of the new kernel, k = rep, rep + R, ... below nseg, against positions
// m < MP of this lane's slot.  A new write conflicts with any intersecting
// segment, a new read only with an intersecting write.  Positions a slot
// does not use hold the empty range [0, 0), which intersects nothing, so MP
// only has to cover the segment counts of the occupied slots.  UNI: nseg is
// the same on every lane (one window), so the loop test is scalar.
template <int MP, bool UNI>
__device__ __forceinline__ uint64_t pair_hits(const DevDesc *d, uint32_t nseg, uint32_t wb, uint32_t R, uint32_t rep,
                                              const uint64_t (&ss)[kSegs], const uint64_t (&se)[kSegs],
                                              const uint64_t (&wmask)[kSegs])
{
    uint64_t hits = 0;
    for (uint32_t k0 = 0; UNI ? k0 < nseg : __builtin_amdgcn_ballot_w64(rep < R && k0 + rep < nseg) != 0; k0 += R) {
        const uint32_t k = k0 + rep;
        const bool kin = rep < R && k < nseg;
        const uint32_t kk = kin ? k : 0u;
        const uint64_t a0 = kin ? d->s[kk] : 0ull, a1 = kin ? d->e[kk] : 0ull;
        // lanes whose new range is a write: they match any slot range
        const uint64_t wkm = __builtin_amdgcn_ballot_w64(kin && ((wb >> kk) & 1u));
        // no branch per position: on the window wave a branch costs more than
        // the two compares it would skip.  The compares go straight into lane
        // masks; the rest is scalar.
#pragma unroll
        for (int m = 0; m < MP; m++)
            hits |= __builtin_amdgcn_ballot_w64(a0 < se[m]) & __builtin_amdgcn_ballot_w64(a1 > ss[m]) & (wkm | wmask[m]);
    }
    return hits;
}

// Slots of the mask `cand` (one group) whose kernels the kernel with group
// sequence number g and upstream list (hup, hup2) depends on (bit b of hup:
// the kernel g - 1 - b; bit b of hup2: the kernel g - 65 - b).  Each lane
// tests the kernel of its own slot.
__device__ __forceinline__ uint64_t slots_upstream(uint64_t cand, uint32_t myg, uint32_t g, uint64_t hup, uint64_t hup2,
                                                   uint32_t lane)
{
    const uint32_t back = g - 1u - myg;
    const uint64_t word = back < 64u ? hup : hup2;
    return __builtin_amdgcn_ballot_w64(((cand >> lane) & 1ull) && back < 128u && ((word >> (back & 63u)) & 1ull));
}

// Largest of x over the wave (x < 2^31): an inclusive running maximum by DPP
// row shifts and row broadcasts (the prefix-sum pattern), read at lane 63.
__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    int32_t m = (int32_t)x, o;
    o = __builtin_amdgcn_update_dpp(0, m, 0x111, 0xf, 0xf, false);   // row_shr:1
    m = o > m ? o : m;
    o = __builtin_amdgcn_update_dpp(0, m, 0x112, 0xf, 0xf, false);   // row_shr:2
    m = o > m ? o : m;
    o = __builtin_amdgcn_update_dpp(0, m, 0x114, 0xf, 0xf, false);   // row_shr:4
    m = o > m ? o : m;
    o = __builtin_amdgcn_update_dpp(0, m, 0x118, 0xf, 0xf, false);   // row_shr:8
    m = o > m ? o : m;
    o = __builtin_amdgcn_update_dpp(0, m, 0x142, 0xa, 0xf, false);   // row_bcast:15
    m = o > m ? o : m;
    o = __builtin_amdgcn_update_dpp(0, m, 0x143, 0xc, 0xf, false);   // row_bcast:31
    m = o > m ? o : m;
    return (uint32_t)__builtin_amdgcn_readlane(m, 63);
}

template <int NG>
__device__ inline void window_wave(const DevParams &p, FetchShared *fs)
{
    const uint32_t lane = threadIdx.x;
    const int W = p.W, G = p.n_groups;
    const bool tr = p.trace != nullptr;
    ACS_GAS HostCtrl *const ctrl = gp(p.ctrl);
    ACS_GAS DevState *const st = gp(p.st);
    ACS_GAS acs_trace_rec *const trace = gp(p.trace);
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t depth = NG == 1 ? kLdsDescs : lds_depth(G);   // a constant for one window
    // One window with its checks made ahead of it (a check wave or the
    // host): a kernel's upstream list arrives with it and admission needs no
    // pair tests.  The host's list is already in the device ring; a check
    // wave's is in the staged copy only, and the window stores it.
    const bool ahead = NG == 1 && p.host_check > 0;
    const bool store_up = !ahead || p.check_wave != 0;
    const uint32_t M = ahead ? (uint32_t)p.host_check : kSpan;   // admission gate, in group sequence numbers

    // Slots: group g owns lanes [g * Wp, g * Wp + W), Wp = W rounded up to a
    // power of two; span = G * Wp lanes hold slots.  When span < 64 and the
    // window makes the pair tests, the slots' ranges are replicated: lane l
    // holds the ranges of slot lane l mod span, and its replica index l / span
    // selects which of the new kernel's segments it tests, so R replicas
    // divide the pair tests of an insertion by R.  Masks are over slot lanes.
    const uint32_t Wp = W <= 1 ? 1u : (W <= 2 ? 2u : (W <= 4 ? 4u : (W <= 8 ? 8u : (W <= 16 ? 16u : (W <= 32 ? 32u : 64u)))));
    const uint32_t span = Wp * (uint32_t)G;
    const uint32_t R = (64u / span) < (uint32_t)kSegs ? 64u / span : (uint32_t)kSegs;   // replicas in use
    const uint32_t sl = lane % span, rep = lane / span, grp = sl / Wp;   // slot lane, replica, group
    const uint64_t wpmask = Wp >= 64 ? ~0ull : ((1ull << Wp) - 1ull);
    const uint64_t spanmask = span >= 64 ? ~0ull : ((1ull << span) - 1ull);
    const uint64_t wmaskslots = W >= 64 ? ~0ull : ((1ull << W) - 1ull);   // usable slots of a group
    const uint64_t mygroup = (wmaskslots & wpmask) << (grp * Wp);
    uint64_t repmul = 0;   // bit r * span set for every replica r
    for (uint32_t r = 0; r < R; r++) repmul |= 1ull << (r * span);

    // the kernel in this lane's slot (slot lanes only)
    uint32_t myg = 0, mynp = 0;   // group sequence number, pieces
    int32_t mykid = 0;
    uint64_t myseq = 0, myhup = 0;   // submission index (traces), upstream list by distance
    uint64_t myhup2 = 0;             // its second word (distances 65 to 128, checks on the host)
    // pair tests: this lane's slot ranges (replicated), and per position the
    // lanes whose slot range there is a write; unused and free positions hold
    // the empty range [0, 0), which intersects nothing
    uint64_t ss[kSegs], se[kSegs], wmask[kSegs];
#pragma unroll
    for (int m = 0; m < kSegs; m++) ss[m] = se[m] = wmask[m] = 0;
    uint64_t over4 = 0, over2 = 0;   // slots using more than 4 (2) positions

    // wave-uniform state
    uint64_t valid = 0, pub = 0, ev = 0, snap_seen = 0, checks = 0;
    uint32_t head[NG];
    uint64_t retired[NG], published[NG];
#pragma unroll
    for (int g = 0; g < NG; g++) {
        head[g] = 0;
        retired[g] = published[g] = 0;
    }

    if (lane == 0) __hip_atomic_store(&ctrl->alive, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);

    for (uint32_t iter = 1;; iter++) {
        bool progress = false;
        if ((iter & 4095u) == 0 && uni32(LDS_LOAD(&fs->stop)) == 2u) break;   // abort is honoured even while busy

        // The completion words of the occupied slots are polled first and
        // examined after admission, so that the load's latency overlaps the
        // admission work.  Read relaxed: the window wave reads no task
        // results, and the workers acquire before their bodies start.
        const bool occ = (valid >> lane) & 1ull;
        const uint32_t cdone =
            occ ? __hip_atomic_load(&st->dseq[grp][myg & (kSeqRing - 1u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;

        // ---- admission in program order (per group), strictly FIFO
        uint32_t ftail[NG];
#pragma unroll
        for (int g = 0; g < NG; g++) ftail[g] = g < G ? uni32(LDS_LOAD(&fs->tail[g])) : 0u;
        bool staged = false;
#pragma unroll
        for (int g = 0; g < NG; g++) staged |= g < G && head[g] != ftail[g];
        uint64_t newly = 0;    // slots admitted now; all of them are handed out below
        bool drain = false;    // upstream lists were stored into the device ring
        if (staged) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (NG == 1 && ahead) {
                // every staged kernel that finds a free slot, at once: the
                // r-th free slot (lane order) takes staged kernel head + r
                const uint64_t freem = ~valid & wmaskslots;
                uint32_t K = (uint32_t)__builtin_popcountll(freem);
                const uint32_t nst = ftail[0] - head[0];
                K = nst < K ? nst : K;
                {
                    // the gate of the split (Section IV-C): kernel head + r
                    // waits while the window holds one more than M older,
                    // counting the kernels admitted before it in this pass
                    // (with an empty window the first of them is the oldest)
                    const uint32_t oldest_back = (valid && K) ? wave_max(occ ? head[0] - myg : 0u) : 0u;
                    const uint32_t room = oldest_back <= M ? M - oldest_back + 1u : 0u;
                    K = room < K ? room : K;
                }
                if (K) {
                    const uint32_t r = (uint32_t)__builtin_popcountll(freem & lane_lt);
                    const bool take = ((freem >> lane) & 1ull) && r < K;
                    newly = __builtin_amdgcn_ballot_w64(take);
                    if (take) {
                        const DevDesc *d = &fs->ring[(head[0] + r) & (depth - 1u)];
                        myseq = d->seq;
                        mykid = d->kid;
                        const uint32_t npr = d->npieces;
                        mynp = npr < kMaxPieces ? (npr ? npr : 1u) : kMaxPieces;
                        myhup = d->host_up;
                        myhup2 = d->host_up_hi;
                        myg = head[0] + r;
                        if (store_up && myhup != 0)
                            __hip_atomic_store(reinterpret_cast<ACS_GAS uint64_t *>(&st->dring[0][myg & (kDescRing - 1u)].host_up),
                                               myhup, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    drain = store_up && __builtin_amdgcn_ballot_w64(take && myhup != 0) != 0;
                    if (tr) {
                        // the upstream slots at each insert, from the lists
                        uint32_t k = 0;
                        for (uint64_t m = newly; m; m &= m - 1, k++) {
                            const int s = __builtin_ctzll(m);
                            const uint64_t vin = valid | (newly & ((1ull << s) - 1ull));
                            const uint64_t upm =
                                slots_upstream(vin, myg, readlane32(myg, s), readlane64(myhup, s), readlane64(myhup2, s), lane);
                            const uint64_t sq = readlane64(myseq, s);
                            const int32_t kd = (int32_t)readlane32((uint32_t)mykid, s);
                            if (lane == 0 && sq < p.trace_cap) trace_insert(&trace[sq], sq, s, kd, ev + k, vin, upm);
                        }
                    }
                    ev += K;
                    valid |= newly;
                    head[0] += K;
                    progress = true;
                }
            } else if constexpr (NG == 1) {
                // checks at insert (Algorithm 1 both ways), one kernel per step;
                // the descriptor is read once by the whole wave (lane i holds
                // its 4-byte word i) and its fields are taken with readlane
                const uint64_t full = wmaskslots & wpmask;
                for (uint32_t pass = 0; pass < kAdmitBatch && head[0] != ftail[0] && valid != full; pass++) {
                    const uint32_t gq = head[0];
                    // a kernel more than kSpan older still in the window: wait
                    if (__builtin_amdgcn_ballot_w64(((valid >> lane) & 1ull) && gq - myg > M) != 0) break;
                    const DevDesc *d = &fs->ring[gq & (depth - 1u)];
                    const uint32_t dw = reinterpret_cast<const uint32_t *>(d)[lane];
                    const int slot = __builtin_ctzll(~valid & full);
                    const uint64_t bit = 1ull << slot;
                    const uint32_t nraw = readlane32(dw, kNsegDword);
                    const uint32_t nseg = nraw < (uint32_t)kSegs ? nraw : (uint32_t)kSegs;
                    const uint32_t wb = readlane32(dw, kWbitsDword);
                    uint64_t hits;
                    if (valid & over4) hits = pair_hits<8, true>(d, nseg, wb, R, rep, ss, se, wmask);
                    else if (valid & over2) hits = pair_hits<4, true>(d, nseg, wb, R, rep, ss, se, wmask);
                    else hits = pair_hits<2, true>(d, nseg, wb, R, rep, ss, se, wmask);
                    uint64_t upm = 0;
                    for (uint32_t r = 0; r < R; r++) upm |= (hits >> (r * span)) & spanmask;
                    upm &= valid;
                    // the same conflicts as an upstream list by distance
                    uint64_t hup = 0;
                    for (uint64_t m = upm; m; m &= m - 1) hup |= 1ull << ((gq - 1u - readlane32(myg, __builtin_ctzll(m))) & 63u);
                    if (hup != 0) {
                        if (lane == 0)
                            __hip_atomic_store(reinterpret_cast<ACS_GAS uint64_t *>(&st->dring[0][gq & (kDescRing - 1u)].host_up), hup,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        drain = true;
                    }
                    if (sl == (uint32_t)slot && rep < R) {
#pragma unroll
                        for (int m = 0; m < kSegs; m++) {
                            ss[m] = d->s[m];
                            se[m] = d->e[m];
                        }
                    }
                    checks += (uint64_t)__builtin_popcountll(valid) * nseg * kSegs;
                    const uint64_t seq = readpair(dw, 0);
                    const int32_t kid = (int32_t)readlane32(dw, kKidDword);
                    const uint32_t npr = readlane32(dw, kNpiecesDword);
                    if ((int)lane == slot) {
                        myseq = seq;
                        mykid = kid;
                        mynp = npr < kMaxPieces ? (npr ? npr : 1u) : kMaxPieces;
                        myg = gq;
                        myhup = hup;
                        myhup2 = 0;
                    }
                    const uint64_t rbit = bit * repmul;
#pragma unroll
                    for (int m = 0; m < kSegs; m++)
                        wmask[m] = ((uint32_t)m < nseg && ((wb >> m) & 1u)) ? (wmask[m] | rbit) : (wmask[m] & ~rbit);
                    over4 = nseg > 4u ? (over4 | bit) : (over4 & ~bit);
                    over2 = nseg > 2u ? (over2 | bit) : (over2 & ~bit);
                    if (tr && lane == 0 && seq < p.trace_cap) trace_insert(&trace[seq], seq, slot, kid, ev, valid, upm);
                    ev++;
                    valid |= bit;
                    newly |= bit;
                    head[0]++;
                    progress = true;
                }
            } else {
                for (uint32_t pass = 0; pass < kAdmitBatch; pass++) {
                    // which groups admit in this step, and into which slot
                    // lane: a group with a staged kernel, a free slot and no
                    // kernel more than kSpan older than it in its window
                    uint32_t hg = 0;
#pragma unroll
                    for (int g = 0; g < NG; g++)
                        if ((uint32_t)g == grp) hg = head[g];
                    const uint64_t gbad = __builtin_amdgcn_ballot_w64(((valid >> lane) & 1ull) && hg - myg > M);
                    uint32_t adm = 0;
                    uint32_t newl[NG];
#pragma unroll
                    for (int g = 0; g < NG; g++) {
                        newl[g] = 0;
                        const uint64_t gm = (wmaskslots & wpmask) << (g * Wp);
                        if (g < G && head[g] != ftail[g] && (gbad & gm) == 0) {
                            const uint64_t fr = ~valid & gm;
                            if (fr) {
                                adm |= 1u << g;
                                newl[g] = (uint32_t)__builtin_ctzll(fr);
                            }
                        }
                    }
                    if (!adm) break;
                    // this lane's group: does it admit, from which staged
                    // descriptor, into which lane
                    const bool gin = (adm >> grp) & 1u;
                    uint32_t nsel = 0;
#pragma unroll
                    for (int g = 0; g < NG; g++)
                        if ((uint32_t)g == grp) nsel = newl[g];
                    const DevDesc *d = &fs->ring[grp * depth + (hg & (depth - 1u))];
                    uint64_t newbits = 0;
#pragma unroll
                    for (int g = 0; g < NG; g++)
                        if ((adm >> g) & 1u) newbits |= 1ull << newl[g];
                    const uint32_t nraw = gin ? d->nseg : 0u;
                    const uint32_t nseg = nraw < (uint32_t)kSegs ? nraw : (uint32_t)kSegs;
                    const uint32_t wb = d->wbits;
                    // segment k of each group's new kernel against every
                    // occupied slot of the group; replica r takes k = r, r + R, ...
                    uint64_t hits;
                    if (valid & over4) hits = pair_hits<8, false>(d, nseg, wb, R, rep, ss, se, wmask);
                    else if (valid & over2) hits = pair_hits<4, false>(d, nseg, wb, R, rep, ss, se, wmask);
                    else hits = pair_hits<2, false>(d, nseg, wb, R, rep, ss, se, wmask);
                    // fold the replicas onto their slot lanes; a new slot's own
                    // lanes may already hold its ranges: only occupied slots count
                    uint64_t upall = 0;
                    for (uint32_t r = 0; r < R; r++) upall |= (hits >> (r * span)) & spanmask;
                    upall &= valid;
                    checks += (uint64_t)__builtin_popcountll(valid) * kSegs * kSegs;
                    // each admitted group's conflicts as an upstream list by distance
                    uint64_t hupl = 0;   // this lane's group's list
#pragma unroll
                    for (int g = 0; g < NG; g++) {
                        if (!((adm >> g) & 1u)) continue;
                        const uint64_t gm = (wmaskslots & wpmask) << (g * Wp);
                        const uint32_t gq = head[g];
                        uint64_t hup = 0;
                        for (uint64_t m = upall & gm; m; m &= m - 1)
                            hup |= 1ull << ((gq - 1u - readlane32(myg, __builtin_ctzll(m))) & 63u);
                        if (hup != 0) {
                            if (lane == 0)
                                __hip_atomic_store(
                                    reinterpret_cast<ACS_GAS uint64_t *>(&st->dring[g][gq & (kDescRing - 1u)].host_up), hup,
                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            drain = true;
                        }
                        if ((uint32_t)g == grp) hupl = hup;
                    }
                    if (gin && sl == nsel && rep < R) {
                        // the new occupant's ranges, in every replica of its slot
#pragma unroll
                        for (int m = 0; m < kSegs; m++) {
                            ss[m] = d->s[m];
                            se[m] = d->e[m];
                        }
                    }
                    if (gin && lane == nsel) {
                        myseq = d->seq;
                        mykid = d->kid;
                        const uint32_t npr = d->npieces;
                        mynp = npr < kMaxPieces ? (npr ? npr : 1u) : kMaxPieces;
                        myg = hg;
                        myhup = hupl;
                        myhup2 = 0;
                        if (tr && myseq < p.trace_cap) {
                            const uint64_t rank = (uint64_t)__builtin_popcount(adm & ((1u << grp) - 1u));
                            trace_insert(&trace[myseq], myseq, (int32_t)lane, mykid, ev + rank, valid & mygroup,
                                         upall & mygroup);
                        }
                    }
                    // write flags of the new occupants' ranges, for every replica
                    // lane of a new slot at once
                    {
                        const bool newrep = gin && sl == nsel && rep < R;
                        const uint64_t newlanes = __builtin_amdgcn_ballot_w64(newrep);
#pragma unroll
                        for (int m = 0; m < kSegs; m++) {
                            const uint64_t wr = __builtin_amdgcn_ballot_w64(newrep && (uint32_t)m < nseg && ((wb >> m) & 1u));
                            wmask[m] = (wmask[m] & ~newlanes) | wr;
                        }
                        const uint64_t big4 = __builtin_amdgcn_ballot_w64(newrep && rep == 0 && nseg > 4u);
                        const uint64_t big2 = __builtin_amdgcn_ballot_w64(newrep && rep == 0 && nseg > 2u);
                        over4 = (over4 & ~newbits) | big4;
                        over2 = (over2 & ~newbits) | big2;
                    }
#pragma unroll
                    for (int g = 0; g < NG; g++)
                        if ((adm >> g) & 1u) head[g]++;
                    ev += (uint64_t)__builtin_popcount(adm);
                    valid |= newbits;
                    newly |= newbits;
                    progress = true;
                }
            }
            // all lanes are done reading the staged descriptors before their
            // LDS slots are handed back to the FIFO wave
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) {
#pragma unroll
                for (int g = 0; g < NG; g++)
                    if (g < G) LDS_STORE(&fs->head[g], head[g]);
            }
        }

        // ---- completions: a slot whose kernel stored its word is free again.
        // Examined before this pass's work-queue stores are issued: waiting
        // for the poll waits for every older memory operation of the wave,
        // and the stores of the previous pass have had the admission work to
        // complete, while this pass's would still be on their way to memory.
        // Slots admitted in this pass were free when the poll was issued, so
        // none of them is among those found complete.
        {
            const uint64_t done = __builtin_amdgcn_ballot_w64(occ && (int32_t)(cdone - (myg + 1u)) >= 0);
            if (done) {
                if (tr) {
                    const uint64_t now = wall_clock64();
                    if (((done >> lane) & 1ull) && myseq < p.trace_cap) {
                        tput(&trace[myseq].ev_retire, (int64_t)(ev + __builtin_popcountll(done & lane_lt)));
                        tput(&trace[myseq].t_retire, (int64_t)now);
                    }
                }
                ev += (uint64_t)__builtin_popcountll(done);
#pragma unroll
                for (int g = 0; g < NG; g++)
                    if (g < G) retired[g] += (uint64_t)__builtin_popcountll(done & (wpmask << (g * Wp)));
                if (!ahead) {
                    if (((done >> sl) & 1ull) && rep < R) {
#pragma unroll
                        for (int m = 0; m < kSegs; m++) ss[m] = se[m] = 0;
                    }
                    const uint64_t rdone = done * repmul;
#pragma unroll
                    for (int m = 0; m < kSegs; m++) wmask[m] &= ~rdone;
                }
                valid &= ~done;
                progress = true;
            }
        }

        // ---- dispatch.  Every admitted kernel is handed out at once: its
        // workers wait for the completion words of the kernels in its
        // upstream list themselves.  Entries are published in admission
        // order (lane order within a pass), so every upstream kernel's
        // entries precede its dependents' in the queue: a worker only ever
        // waits for work that an earlier ticket holds.
        if (newly) {
            // the upstream lists stored above are complete before any entry
            // that points at them, and so are the trace records' initial
            // values (else a worker's update of the record could land first
            // and be overwritten).  0x0F70: vmcnt 0, expcnt 7, lgkmcnt 15.
            if (drain || tr) __builtin_amdgcn_s_waitcnt(0x0F70);
            const bool mine = (newly >> lane) & 1ull;
            int32_t total;
            const uint32_t before = (uint32_t)wave_exclusive_scan(mine ? (int32_t)mynp : 0, &total);
            // a kernel of one piece: its own lane writes the entry (one store
            // for all of them); a kernel of several: the whole wave does
            if (mine && mynp == 1) {
                const uint64_t t = pub + before;
                __hip_atomic_store(&st->ent[t & (kQueueCap - 1)], queue_entry(t, grp, 0, myg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            for (uint64_t m = __builtin_amdgcn_ballot_w64(mine && mynp > 1); m; m &= m - 1) {
                const int l = __builtin_ctzll(m);
                const uint32_t bl = readlane32(before, l), nl = readlane32(mynp, l), gl = readlane32(myg, l);
                const uint32_t grl = (uint32_t)l / Wp;
                for (uint32_t q = lane; q < nl; q += kWave) {
                    const uint64_t t = pub + bl + q;
                    __hip_atomic_store(&st->ent[t & (kQueueCap - 1)], queue_entry(t, grl, q, gl), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (tr && mine && myseq < p.trace_cap) {
                tput(&trace[myseq].ev_dispatch, (int64_t)(ev + __builtin_popcountll(newly & lane_lt)));
                tput(&trace[myseq].t_dispatch, (int64_t)wall_clock64());
            }
            pub += (uint64_t)(uint32_t)total;
            ev += (uint64_t)__builtin_popcountll(newly);
        }

        // ---- the host learns about completions when a group drains: one
        // system-scope release covers every result (and trace record) of the
        // kernels retired so far
        uint32_t drained = 0;
#pragma unroll
        for (int g = 0; g < NG; g++)
            if (g < G && (valid & (wpmask << (g * Wp))) == 0 && retired[g] != published[g]) drained |= 1u << g;
        if (drained) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
#pragma unroll
            for (int g = 0; g < NG; g++)
                if ((drained >> g) & 1u) {
                    if (lane == 0)
                        __hip_atomic_store(&ctrl->retired[g], retired[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    published[g] = retired[g];
                }
        }

        if (!progress) {
            // snapshot of the window for the host (the scheduled list): the
            // upstream slots of each kernel from its list; every kernel in the
            // window has been handed out, so it is executing unless it still
            // waits for an upstream kernel
            const uint64_t sr = uni64(LDS_LOAD(&fs->snap_req));
            if (sr != snap_seen) {
                uint64_t myup = 0;
                for (uint64_t m = valid; m; m &= m - 1) {
                    const int s = __builtin_ctzll(m);
                    const uint64_t gm = (wmaskslots & wpmask) << (((uint32_t)s / Wp) * Wp);
                    const uint64_t u =
                        slots_upstream(valid & gm, myg, readlane32(myg, s), readlane64(myhup, s), readlane64(myhup2, s), lane);
                    if ((int)lane == s) myup = u;
                }
                const bool v = (valid >> lane) & 1ull;
                uint32_t rank = 0;
                for (uint64_t m = valid; m; m &= m - 1) {
                    const int l = __builtin_ctzll(m);
                    rank += (readlane64(myseq, l) < myseq) ? 1u : 0u;
                }
                if (v) {
                    acs_entry e;
                    e.seq = myseq;
                    e.kernel_id = mykid;
                    e.state = myup != 0 ? ACS_PENDING : ACS_EXECUTING;
                    e.upstream_mask = myup;
                    e.slot = (int32_t)lane;
                    e.reserved = 0;
                    ctrl->snap[rank] = e;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                if (lane == 0) {
                    __hip_atomic_store(&ctrl->snap_count, (uint64_t)__builtin_popcountll(valid), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&ctrl->snap_ack, sr, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                snap_seen = sr;
            }
            const uint32_t stp = uni32(LDS_LOAD(&fs->stop));
            bool empty = valid == 0;
#pragma unroll
            for (int g = 0; g < NG; g++) empty &= g >= G || head[g] == uni32(LDS_LOAD(&fs->tail[g]));
            if (stp == 2u || (stp == 1u && empty)) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }

    // leave: stop the FIFO wave and give every worker an exit entry
    if (lane == 0) LDS_STORE(&fs->exit, 1u);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (uint32_t i = lane; i < (uint32_t)p.n_workers; i += 64) {
        const uint64_t t = pub + i;
        __hip_atomic_store(&st->ent[t & (kQueueCap - 1)], queue_entry(t, kSentinelGroup, 0, 0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
        __hip_atomic_store(&ctrl->checks, checks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&ctrl->published, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&ctrl->exited, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__device__ inline void worker(const DevParams &p, uint8_t *smem, Mail *mail)
{
    // Control flow here is uniform across each wave by construction: wave 0
    // (selected through readfirstlane, so the compiler sees a uniform branch)
    // claims tickets and reports completions with all 64 lanes active, and
    // every value that decides a branch is taken from the first lane.  A
    // lane-divergent region next to the workgroup barriers of this loop can
    // be compiled into a loop that re-enters the barrier without the lanes of
    // that region, which never terminates.
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const bool wave0 = uni32(tid) < 64u;
    const bool tr = p.trace != nullptr;
    ACS_GAS HostCtrl *const ctrl = gp(p.ctrl);
    ACS_GAS DevState *const st = gp(p.st);
    ACS_GAS acs_trace_rec *const trace = gp(p.trace);
    uint64_t *margs = reinterpret_cast<uint64_t *>(mail->args);
    for (;;) {
        if (wave0) {
            // every lane adds 1, so one ticket is kWave counts of deq: with a
            // value the same on all lanes the compiler issues one atomic and
            // a popcount, where a per-lane value costs a loop over the lanes
            // (the host checks the final count after the kernel exits)
            const uint64_t t = uni64(__hip_atomic_fetch_add(&st->deq, 1ull, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)) / kWave;
            const uint64_t tag = ((t >> 16) + 1u) & 0xFFu;
            uint64_t v;
            for (uint32_t spin = 1;; spin++) {
                v = uni64(__hip_atomic_load(&st->ent[t & (kQueueCap - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if ((v >> 56) == tag) break;
                // a host abort releases waiting workers even if the window wave has left
                if ((spin & 1023u) == 0 &&
                    uni64(__hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) == 2ull) {
                    v = (uint64_t)kSentinelGroup << 48;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t grp = (uint32_t)(v >> 48) & 0xFFu, g = (uint32_t)v;
            // all lanes store the same values: no lane-divergent branch needed
            mail->group = grp;
            mail->piece = (uint32_t)(v >> 32) & 0xFFFFu;
            mail->gseq = g;
            if (grp != kSentinelGroup) {
                const ACS_GAS DevDesc *te = &st->dring[grp][g & (kDescRing - 1u)];
                mail->kid = te->kid;
                const uint32_t npr = te->npieces;
                mail->np = npr < kMaxPieces ? (npr ? npr : 1u) : kMaxPieces;
                mail->seq = te->seq;
                margs[lane & 7u] = reinterpret_cast<const ACS_GAS uint64_t *>(te->args)[lane & 7u];
                // wait until every upstream kernel has stored its completion
                // word (lane b watches the kernel b + 1 places back and, with
                // the second word, the kernel b + 65 places back)
                const uint64_t hup = uni64(te->host_up);
                const uint64_t hup2 = uni64(te->host_up_hi);
                if ((hup | hup2) != 0) {
                    const bool watch = (hup >> lane) & 1ull, watch2 = (hup2 >> lane) & 1ull;
                    const uint32_t k = g - 1u - lane, k2 = g - 65u - lane;
                    for (uint32_t spin = 1;; spin++) {
                        bool ok = true;
                        if (watch) {
                            const uint32_t c =
                                __hip_atomic_load(&st->dseq[grp][k & (kSeqRing - 1u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            ok = (int32_t)(c - (k + 1u)) >= 0;
                        }
                        if (hup2 != 0 && watch2) {
                            const uint32_t c =
                                __hip_atomic_load(&st->dseq[grp][k2 & (kSeqRing - 1u)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            ok = ok && (int32_t)(c - (k2 + 1u)) >= 0;
                        }
                        if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
                        if ((spin & 1023u) == 0 &&
                            uni64(__hip_atomic_load(&ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) == 2ull)
                            break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                if (tr) mail->t0 = uni64(wall_clock64());
            }
        }
        __syncthreads();
        const uint32_t grp = uni32(mail->group);
        if (grp == kSentinelGroup) break;
        // read before the barrier below: past it, wave 0 may take the next
        // ticket and rewrite the mail
        const uint32_t kid = uni32((uint32_t)mail->kid);
        run_body<true>((int32_t)kid, mail->args, uni32(mail->piece), uni32(mail->np), smem);
        // each wave waits until its own result stores (device scope) are
        // complete, so that they are visible device-wide before wave 0 counts
        // the piece (the workgroup barrier alone waits only for LDS traffic).
        // 0x0F70: vmcnt 0, expcnt 7, lgkmcnt 15.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        if (wave0) {
            const uint64_t seq = uni64(mail->seq);
            if (tr && seq < p.trace_cap) {
                // one lane: 64 read-modify-writes of one address would queue
                // behind each other before the completion store below
                const uint64_t t1 = uni64(wall_clock64()), t0 = uni64(mail->t0);
                if (lane == 0) {
                    __hip_atomic_fetch_min(reinterpret_cast<ACS_GAS uint64_t *>(&trace[seq].t_start), t0, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_max(reinterpret_cast<ACS_GAS uint64_t *>(&trace[seq].t_end), t1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            // a kernel of several pieces is complete when the last piece is
            // counted; every piece's results were complete before its count,
            // so the last count comes after all of them.  The last piece
            // resets the counter for the next kernel at this ring place
            // (which cannot be admitted before this one's word is seen).
            const uint32_t np = uni32(mail->np), g = uni32(mail->gseq);
            bool last = true;
            if (np > 1) {
                // every lane adds 1: a piece counts kWave (see the ticket above)
                const uint32_t old = uni32(__hip_atomic_fetch_add(&st->cnt[grp][g & (kSeqRing - 1u)], 1u, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT));
                last = old + kWave == kWave * np;
                if (last) {
                    __hip_atomic_store(&st->cnt[grp][g & (kSeqRing - 1u)], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_s_waitcnt(0x0F70);
                }
            }
            if (last)
                __hip_atomic_store(&st->dseq[grp][g & (kSeqRing - 1u)], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // an islands kernel's plan goes to the host only now (plan_publish),
        // before the body scratch that holds it is used again; every wave
        // takes this branch or none (kid was read before the barrier), and
        // wave 0 rewrites the mail only after it
        if (kid == (uint32_t)ACS_K_RL_ISLANDS) {
            __syncthreads();
            plan_publish(load_args<acs_args_rl>(mail->args), smem);
        }
    }
}

}  // namespace acs
