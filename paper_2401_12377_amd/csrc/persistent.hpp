// Wave-level building blocks of the persistent scheduler kernel (device code).
//
// Workgroup 0 is the window:
//   wave 0  the window module.  Lane i owns window slot i: its read/write
//           ranges, its upstream bitmask and its completion target live in
//           that lane's registers.  Inserting a kernel is one pass in which
//           every lane tests the new kernel's ranges against its own slot
//           (Algorithm 1, both directions) and a ballot gives the new
//           kernel's upstream mask.  Completions are seen by polling the
//           per-slot completion counters; a ballot of finished slots clears
//           those bits in every lane's mask at once.  The ready mask is a
//           ballot of (valid, not executing, empty upstream mask); ready
//           kernels are published, oldest first, as (slot, piece) entries of a
//           work queue in device memory.
//   wave 1  the input FIFO: copies descriptors from the host-resident ring
//           into a small ring in LDS, so that host-memory latency never
//           stalls the window loop.
// Workgroups 1.. are workers: each takes a ticket from the work queue, waits
// for the entry with that ticket, runs one piece of the task body, and bumps
// the slot's completion counter with release semantics.
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

constexpr uint32_t kLdsRing = 16;   // descriptors staged in LDS
constexpr uint32_t kAdmitBatch = 16; // insertions per pass of the window loop while workers are busy
constexpr uint32_t kAdmitFew = 2;     // ... and while fewer than kBusyKernels kernels are out
constexpr uint32_t kBusyKernels = 4;

struct FetchShared {
    uint32_t tail;       // descriptors staged (written by the FIFO wave)
    uint32_t head;       // descriptors taken (written by the window wave)
    uint32_t stop;       // mirror of the host stop flag
    uint32_t exit;       // window wave -> FIFO wave: leave
    uint64_t snap_req;   // mirror of the host snapshot request counter
    uint64_t pad;
    DevDesc ring[kLdsRing];
};
static_assert(sizeof(FetchShared) <= kBodySmem, "FIFO staging must fit the LDS scratch");

struct Mail {
    uint32_t slot, piece;
    int32_t kid;
    uint32_t np, ptarget, pad;
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

__device__ inline void fifo_wave(const DevParams &p, FetchShared *fs)
{
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t consumed = 0, htail = 0;
    uint32_t ftail = 0;
    bool idle = true;
    for (;;) {
        if (uni32(LDS_LOAD(&fs->exit))) break;
        const uint32_t head = uni32(LDS_LOAD(&fs->head));
        const uint32_t space = kLdsRing - (ftail - head);
        bool moved = false;
        uint64_t st = 0;
        if (consumed == htail || idle) {
            // the host's line holds tail, stop and the snapshot request: the three
            // loads are issued together, one round trip to host memory
            const uint64_t t = __hip_atomic_load(&p.ctrl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const uint64_t s0 = __hip_atomic_load(&p.ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const uint64_t sr = __hip_atomic_load(&p.ctrl->snap_req, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            htail = uni64(t);
            st = uni64(s0);
            const uint64_t sru = uni64(sr);
            if (lane == 0) {
                LDS_STORE(&fs->stop, (uint32_t)st);
                LDS_STORE(&fs->snap_req, sru);
            }
            if (htail != consumed) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        }
        if (space > 0) {
            const uint64_t avail = htail - consumed;
            const uint32_t n = avail < space ? (uint32_t)avail : space;
            if (n > 0) {
                // 16 bytes per lane per row, up to 4 rows (16 descriptors).  Rows
                // past the end re-read the last published descriptor (always
                // valid memory) and are not stored.
                uint4 v[4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    uint32_t off = (r * 64u + lane) * 16u;
                    if (off >= n * 256u) off = (n - 1) * 256u + (off % 256u);
                    const uint32_t d = off / 256u, w = off % 256u;
                    const char *src = reinterpret_cast<const char *>(&p.ring[(consumed + d) & p.ring_mask]) + w;
                    v[r] = *reinterpret_cast<const uint4 *>(src);
                }
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const uint32_t off = (r * 64u + lane) * 16u;
                    if (off < n * 256u) {
                        const uint32_t d = off / 256u, w = off % 256u;
                        char *dst = reinterpret_cast<char *>(&fs->ring[(ftail + d) % kLdsRing]) + w;
                        *reinterpret_cast<uint4 *>(dst) = v[r];
                    }
                }
                // every lane's part of the copy lands before lane 0 publishes it
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                ftail += n;
                consumed += n;
                if (lane == 0) {
                    LDS_STORE(&fs->tail, ftail);
                    __hip_atomic_store(&p.ctrl->consumed, consumed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                moved = true;
            }
        }
        idle = !moved;
        if (!moved) {
            if (st == 2) break;   // host abort: leave even if the window wave is gone
            __builtin_amdgcn_s_sleep(1);
        }
    }
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

__device__ inline void window_wave(const DevParams &p, FetchShared *fs)
{
    const uint32_t lane = threadIdx.x;
    const int W = p.W;
    const uint64_t full = (W >= 64) ? ~0ull : ((1ull << W) - 1ull);
    const bool tr = p.trace != nullptr;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // Lanes 0..W-1 own the window slots.  When the window is narrower than
    // the wave, the slots' ranges are replicated: with Wp = W rounded up to a
    // power of two, lane l holds the ranges of slot l mod Wp, and its replica
    // index l / Wp selects which of the new kernel's segments it tests, so R
    // replicas divide the pair tests of an insertion by R.
    const uint32_t Wp = W <= 1 ? 1u : (W <= 2 ? 2u : (W <= 4 ? 4u : (W <= 8 ? 8u : (W <= 16 ? 16u : (W <= 32 ? 32u : 64u)))));
    const uint32_t R = (64u / Wp) < (uint32_t)kSegs ? 64u / Wp : (uint32_t)kSegs;   // replicas in use
    const uint32_t rslot = lane & (Wp - 1), rep = lane / Wp;
    const uint64_t wpmask = Wp >= 64 ? ~0ull : ((1ull << Wp) - 1ull);
    uint64_t repmul = 0;   // bit r * Wp set for every replica r
    for (uint32_t r = 0; r < R; r++) repmul |= 1ull << (r * Wp);

    // this lane's slot (rslot; lanes whose replica index is R or more hold nothing)
    uint64_t ss[kSegs], se[kSegs];
#pragma unroll
    for (int m = 0; m < kSegs; m++) ss[m] = se[m] = 0;
    uint32_t target = 0, mynp = 0;
    int32_t mykid = 0;
    uint64_t up = 0, myseq = 0;

    // wave-uniform state
    uint64_t valid = 0, exec = 0, retired = 0, published = 0, pub = 0, ev = 0, snap_seen = 0, checks = 0;
    uint32_t head = 0;
    // wmask[m]: lanes whose slot segment m is a write.  Segments a slot does
    // not use, and every segment of a free slot, are the empty range [0, 0),
    // which intersects nothing, so the pair test needs no occupancy mask.
    uint64_t wmask[kSegs];
#pragma unroll
    for (int m = 0; m < kSegs; m++) wmask[m] = 0;

    if (lane == 0) __hip_atomic_store(&p.ctrl->alive, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);

    for (uint32_t iter = 1;; iter++) {
        bool progress = false;
        if ((iter & 4095u) == 0 && uni32(LDS_LOAD(&fs->stop)) == 2u) break;   // abort is honoured even while busy

        // The completion words are polled first and examined after admission,
        // so that the load's latency overlaps the insertion work.  They are
        // read relaxed; the acquire that pairs with the workers' releases is
        // taken once, just before the host is told (below).
        const bool mine = (exec >> lane) & 1ull;
        const uint32_t cdone = mine ? __hip_atomic_load(&p.st->done[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;

        // ---- admission in program order while a slot is free, a bounded
        // number per pass
        const uint32_t ftail = uni32(LDS_LOAD(&fs->tail));
        if (head != ftail && valid != full) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            // with few kernels out, dispatch soon rather than admit a long run first
            const uint32_t batch = (uint32_t)__builtin_popcountll(exec) < kBusyKernels ? kAdmitFew : kAdmitBatch;
            for (uint32_t budget = batch; head != ftail && valid != full && budget > 0; budget--) {
                const DevDesc *d = &fs->ring[head % kLdsRing];
                // one LDS read brings the whole descriptor into the wave: lane
                // i holds its 4-byte word i; fields are taken with readlane
                const uint32_t dw = reinterpret_cast<const uint32_t *>(d)[lane];
                const int slot = __builtin_ctzll(~valid);
                const uint64_t bit = 1ull << slot;
                const uint32_t nraw = readlane32(dw, 4);
                const uint32_t nseg = nraw < (uint32_t)kSegs ? nraw : (uint32_t)kSegs;
                const uint32_t wb = readlane32(dw, 5);
                const uint64_t seq = readpair(dw, 0);
                const int32_t kid = (int32_t)readlane32(dw, 2);
                const uint32_t npr = readlane32(dw, 3);
                const uint32_t np = npr < kMaxPieces ? npr : kMaxPieces;
                // the descriptor goes to the task table as it is
                if (lane < kDescCopyDwords) reinterpret_cast<uint32_t *>(&p.st->task[slot])[lane] = dw;
                // Algorithm 1 in both directions: segment k of the new kernel
                // against segment m of every occupied slot.  A new write
                // conflicts with any intersecting segment, a new read only with
                // an intersecting write.  Replica r takes k = r, r + R, ...;
                // segments past nseg are the empty range and match nothing.
                uint64_t hits = 0;
                for (uint32_t k0 = 0; k0 < nseg; k0 += R) {
                    const uint32_t k = k0 + rep;
                    const bool kin = rep < R && k < nseg;
                    const uint32_t kk = kin ? k : 0u;
                    const uint64_t a0 = kin ? d->s[kk] : 0ull, a1 = kin ? d->e[kk] : 0ull;
                    // lanes whose new range is a write: they match any slot range
                    const uint64_t wkm = __builtin_amdgcn_ballot_w64(kin && ((wb >> kk) & 1u));
                    // all eight positions, no branch: unused positions hold the empty
                    // range; on the window wave a branch per position costs more than
                    // the two compares it would skip.  The compares go straight into
                    // lane masks; the rest is scalar.
#pragma unroll
                    for (int m = 0; m < kSegs; m++)
                        hits |= __builtin_amdgcn_ballot_w64(a0 < se[m]) & __builtin_amdgcn_ballot_w64(a1 > ss[m]) &
                                (wkm | wmask[m]);
                }
                // fold the replicas' lanes onto their slots; the new slot's own
                // lanes may already hold its ranges: only occupied slots count
                uint64_t upm = 0;
                for (uint32_t r = 0; r < R; r++) upm |= (hits >> (r * Wp)) & wpmask;
                upm &= valid;
                if (rslot == (uint32_t)slot && rep < R) {
                    // the new occupant's ranges, in every replica of its slot
#pragma unroll
                    for (int m = 0; m < kSegs; m++) {
                        ss[m] = d->s[m];
                        se[m] = d->e[m];
                    }
                }
                checks += (uint64_t)__builtin_popcountll(valid) * nseg * kSegs;
                if ((int)lane == slot) {
                    up = upm;
                    myseq = seq;
                    mykid = kid;
                    mynp = np;
                    if (np > 1) target += np;
                    p.st->task[slot].ptarget = target;
                }
                const uint64_t rbit = bit * repmul;
#pragma unroll
                for (int m = 0; m < kSegs; m++)
                    wmask[m] = ((uint32_t)m < nseg && ((wb >> m) & 1u)) ? (wmask[m] | rbit) : (wmask[m] & ~rbit);
                if (tr && lane == 0 && seq < p.trace_cap) {
                    acs_trace_rec *r = &p.trace[seq];
                    r->seq = (int64_t)seq;
                    r->slot = slot;
                    r->kernel_id = kid;
                    r->ev_insert = (int64_t)ev;
                    r->ev_dispatch = -1;
                    r->ev_retire = -1;
                    r->valid_mask = valid;
                    r->up_mask = upm;
                    r->t_start = INT64_MAX;
                    r->t_end = 0;
                    r->t_dispatch = -1;
                    r->t_retire = -1;
                }
                ev++;
                valid |= bit;
                head++;
                progress = true;
            }
            // all lanes are done reading the staged descriptors before their
            // LDS slots are handed back to the FIFO wave
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) LDS_STORE(&fs->head, head);
        }

        // ---- completions: clear finished slots from every upstream mask
        {
            const uint64_t done = __ballot(mine && (int32_t)(cdone - (uint32_t)(myseq + 1)) >= 0);
            if (done) {
                if (tr) {
                    const uint64_t now = wall_clock64();
                    if (((done >> lane) & 1ull) && myseq < p.trace_cap) {
                        p.trace[myseq].ev_retire = (int64_t)(ev + __builtin_popcountll(done & lane_lt));
                        p.trace[myseq].t_retire = (int64_t)now;
                    }
                }
                ev += __builtin_popcountll(done);
                retired += __builtin_popcountll(done);
                if (((done >> rslot) & 1ull) && rep < R) {
#pragma unroll
                    for (int m = 0; m < kSegs; m++) ss[m] = se[m] = 0;
                }
                const uint64_t rdone = done * repmul;
#pragma unroll
                for (int m = 0; m < kSegs; m++) wmask[m] &= ~rdone;
                up &= ~done;
                valid &= ~done;
                exec &= ~done;
                progress = true;
            }
        }

        // ---- dispatch.  A kernel with an empty upstream mask is ready (it
        // may start at once); a kernel whose upstream kernels have all been
        // handed to the workers is dispatched as well, together with the
        // completion-counter values its workers must see before starting, so
        // that a dependent kernel starts without a round trip through this
        // wave.  Rounds repeat so that a chain inside the window goes out in
        // one pass; entries are published oldest first, so every upstream
        // kernel's work items precede its dependents' in the queue.
        uint64_t newly = 0;
        for (;;) {
            const uint64_t out = exec | newly;
            const bool cand = (((valid & ~out) >> lane) & 1ull) && (up & ~out) == 0;
            const uint64_t r = __ballot(cand);
            if (!r) break;
            newly |= r;
        }
        if (newly) {
            for (uint64_t m = newly; m; m &= m - 1) {
                const int j = __builtin_ctzll(m);
                const uint64_t upj = readlane64(up, j);
                if ((upj >> lane) & 1ull) p.st->wait_target[j][lane] = (uint32_t)(myseq + 1);
                if (lane == 0) p.st->task[j].wait_mask = upj;
            }
            // task-table entries written by other lanes are published before
            // any work-queue entry that points at them
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const bool mine = (newly >> lane) & 1ull;
            uint32_t before = 0, rank = 0, total = 0;
            for (uint64_t m = newly; m; m &= m - 1) {
                const int l = __builtin_ctzll(m);
                const uint64_t sl = readlane64(myseq, l);
                const uint32_t npl = readlane32(mynp, l);
                if (sl < myseq) {
                    before += npl;
                    rank++;
                }
                total += npl;
            }
            if (mine) {
                for (uint32_t q = 0; q < mynp; q++) {
                    const uint64_t t = pub + before + q;
                    const uint64_t v = ((uint64_t)(uint32_t)(t + 1) << 32) | ((uint64_t)lane << 24) | q;
                    __hip_atomic_store(&p.st->ent[t & (kQueueCap - 1)], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                if (tr && myseq < p.trace_cap) {
                    p.trace[myseq].ev_dispatch = (int64_t)(ev + rank);
                    p.trace[myseq].t_dispatch = (int64_t)wall_clock64();
                }
            }
            pub += total;
            ev += __builtin_popcountll(newly);
            exec |= newly;
            progress = true;
        }

        // ---- the host learns about completions when the window drains: one
        // system-scope release covers every result (and trace record) of the
        // kernels retired so far
        if (valid == 0 && retired != published) {
            // pairs with the release of every completion counted so far ...
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_wave_barrier();
            // ... and hands their results on to the host
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
            if (lane == 0) __hip_atomic_store(&p.ctrl->retired, retired, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            published = retired;
        }

        if (!progress) {
            // snapshot of the window for the host (the scheduled list)
            const uint64_t sr = uni64(LDS_LOAD(&fs->snap_req));
            if (sr != snap_seen) {
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
                    e.state = up != 0 ? ACS_PENDING : (((exec >> lane) & 1ull) ? ACS_EXECUTING : ACS_READY);
                    e.upstream_mask = up;
                    e.slot = (int32_t)lane;
                    e.reserved = 0;
                    p.ctrl->snap[rank] = e;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                if (lane == 0) {
                    __hip_atomic_store(&p.ctrl->snap_count, (uint64_t)__builtin_popcountll(valid), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_store(&p.ctrl->snap_ack, sr, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                }
                snap_seen = sr;
            }
            const uint32_t st = uni32(LDS_LOAD(&fs->stop));
            if (st == 2u || (st == 1u && valid == 0 && head == uni32(LDS_LOAD(&fs->tail)))) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }

    // leave: stop the FIFO wave and give every worker an exit entry
    if (lane == 0) LDS_STORE(&fs->exit, 1u);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (uint32_t i = lane; i < (uint32_t)p.n_workers; i += 64) {
        const uint64_t t = pub + i;
        const uint64_t v = ((uint64_t)(uint32_t)(t + 1) << 32) | ((uint64_t)kSentinelSlot << 24);
        __hip_atomic_store(&p.st->ent[t & (kQueueCap - 1)], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
        __hip_atomic_store(&p.ctrl->checks, checks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&p.ctrl->exited, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__device__ inline void worker(const DevParams &p, uint8_t *smem, Mail *mail)
{
    // Control flow here is uniform across each wave by construction: wave 0
    // (selected through readfirstlane, so the compiler sees a uniform branch)
    // claims tickets and reports completions with all 64 lanes active, only
    // lane 0 contributing a non-zero increment, and every value that decides
    // a branch is taken from the first lane.  A lane-divergent region next to
    // the workgroup barriers of this loop can be compiled into a loop that
    // re-enters the barrier without the lanes of that region, which never
    // terminates.
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const bool wave0 = uni32(tid) < 64u;
    const bool tr = p.trace != nullptr;
    uint64_t *margs = reinterpret_cast<uint64_t *>(mail->args);
    for (;;) {
        if (wave0) {
            const uint64_t t = uni64(__hip_atomic_fetch_add(&p.st->deq, lane == 0 ? 1ull : 0ull, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT));
            const uint32_t tag = (uint32_t)(t + 1);
            uint64_t v;
            for (uint32_t spin = 1;; spin++) {
                v = uni64(__hip_atomic_load(&p.st->ent[t & (kQueueCap - 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                if ((uint32_t)(v >> 32) == tag) break;
                // a host abort releases waiting workers even if the window wave has left
                if ((spin & 1023u) == 0 &&
                    uni64(__hip_atomic_load(&p.ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) == 2ull) {
                    v = (uint64_t)kSentinelSlot << 24;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t slot = (uint32_t)(v >> 24) & 0xFFu;
            // all lanes store the same values: no lane-divergent branch needed
            mail->slot = slot;
            mail->piece = (uint32_t)v & 0xFFFFFFu;
            if (slot != kSentinelSlot) {
                const TaskEntry *te = &p.st->task[slot];
                mail->kid = te->kid;
                mail->np = te->npieces;
                mail->ptarget = te->ptarget;
                mail->seq = te->seq;
                margs[lane & 7u] = reinterpret_cast<const uint64_t *>(te->args)[lane & 7u];
                // dispatched early: wait until every upstream kernel's counter
                // has reached the value that marks it complete (lane s watches slot s)
                const uint64_t wm = uni64(te->wait_mask);
                if (wm != 0) {
                    const bool watch = (wm >> lane) & 1ull;
                    const uint32_t tgt = watch ? p.st->wait_target[slot][lane] : 0u;
                    for (uint32_t spin = 1;; spin++) {
                        bool ok = true;
                        if (watch) {
                            const uint32_t c = __hip_atomic_load(&p.st->done[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            ok = (int32_t)(c - tgt) >= 0;
                        }
                        if (__ballot(!ok) == 0) break;
                        if ((spin & 1023u) == 0 &&
                            uni64(__hip_atomic_load(&p.ctrl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) == 2ull)
                            break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                if (tr) mail->t0 = uni64(wall_clock64());
            }
        }
        __syncthreads();
        const uint32_t slot = uni32(mail->slot);
        if (slot == kSentinelSlot) break;
        run_body((int32_t)uni32((uint32_t)mail->kid), mail->args, uni32(mail->piece), uni32(mail->np), smem);
        // each wave waits for its own stores to complete (the workgroup
        // barrier alone waits only for LDS traffic), then wave 0's release
        // below makes every wave's results visible device-wide before the
        // completion counter moves.  0x0F70: vmcnt 0, expcnt 7, lgkmcnt 15.
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        if (wave0) {
            const uint64_t seq = uni64(mail->seq);
            if (tr && seq < p.trace_cap) {
                // one lane: 64 read-modify-writes of one address would queue
                // behind each other before the completion store below
                const uint64_t t1 = uni64(wall_clock64()), t0 = uni64(mail->t0);
                if (lane == 0) {
                    atomicMin(reinterpret_cast<unsigned long long *>(&p.trace[seq].t_start), (unsigned long long)t0);
                    atomicMax(reinterpret_cast<unsigned long long *>(&p.trace[seq].t_end), (unsigned long long)t1);
                }
            }
            // a kernel of several pieces is complete when the last piece is
            // counted; that piece's read-modify-write also acquires the other
            // pieces' results, so its release below covers them
            const uint32_t np = uni32(mail->np);
            bool last = true;
            if (np > 1) {
                const uint32_t old = uni32(__hip_atomic_fetch_add(&p.st->cnt[slot], lane == 0 ? 1u : 0u, __ATOMIC_ACQ_REL,
                                                                  __HIP_MEMORY_SCOPE_AGENT));
                last = old + 1u == uni32(mail->ptarget);
            }
            if (last)
                __hip_atomic_store(&p.st->done[slot], (uint32_t)(seq + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace acs
