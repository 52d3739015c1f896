// CPU build of the persistent scheduler kernel (persistent.hpp, bodies.hpp)
// on top of the built-in emulation in hip/hip_runtime.h of this directory.
// Test infrastructure only.  sim_run() plays both sides: the host submits
// descriptors through the same ring protocol as libacs, and one OS thread
// per GPU thread runs workgroup 0 (window + FIFO waves) and the workers.
#include "hip/hip_runtime.h"

#include <stdlib.h>

#include <chrono>
#include <memory>
#include <thread>
#include <vector>

#include "persistent.hpp"

namespace acs_sim {
thread_local uint32_t tid, bid;
thread_local Group *group;
}  // namespace acs_sim

namespace {
double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Block {
    std::unique_ptr<std::barrier<>> bar;
    acs_sim::Group g;
    alignas(16) uint8_t lds[acs::kBodySmem];
    acs::Mail mail;
};

void run_thread(const acs::DevParams &p, Block *b, uint32_t t, uint32_t blk)
{
    using namespace acs;
    acs_sim::tid = t;
    acs_sim::bid = blk;
    acs_sim::group = &b->g;
    if (blk == 0) {
        FetchShared *fs = reinterpret_cast<FetchShared *>(b->lds);
        if (t == 0) acs::fetch_init(fs);
        __syncthreads();
        const uint32_t wave = acs::uni32(threadIdx.x) >> 6;
        // the smallest compiled group bound that covers the window's groups
        const int32_t ng = p.n_groups;
        if (wave == 0) {
            if (ng <= 1) acs::window_wave<1>(p, fs);
            else if (ng <= 2) acs::window_wave<2>(p, fs);
            else if (ng <= 4) acs::window_wave<4>(p, fs);
            else acs::window_wave<8>(p, fs);
        } else if (wave == 1) {
            if (ng <= 1) acs::fifo_wave<1>(p, fs);
            else if (ng <= 2) acs::fifo_wave<2>(p, fs);
            else if (ng <= 4) acs::fifo_wave<4>(p, fs);
            else acs::fifo_wave<8>(p, fs);
        } else if (wave >= 2 && ng <= 1 && p.check_wave) {
            acs::check_wave(p, fs, wave - 2);
        }
    } else {
        worker(p, b->lds, &b->mail);
    }
    b->bar->arrive_and_drop();
}
}  // namespace

extern "C" {

typedef struct {
    int32_t kid;
    uint32_t npieces, nseg, wbits;
    uint64_t s[8], e[8];
    uint8_t args[64];
} sim_desc;

// Returns 0, or -5 when the window did not retire everything within
// timeout_s (the emulated kernel is then aborted through the stop flag).
// groups[i] (NULL: all 0) is the window group of descriptor i, n_groups the
// number of groups of W slots.
static int run_sim(int32_t W, int32_t n_groups, int32_t host_check, int32_t check_wave, int32_t n_workers, int32_t n,
                   const sim_desc *descs, const int32_t *groups, const uint64_t *host_up, uint32_t ring_cap,
                   acs_trace_rec *trace_out, double timeout_s, uint64_t *retired_out, const uint64_t *host_up_hi = nullptr)
{
    using namespace acs;
    int32_t wp = 1;
    while (wp < W) wp <<= 1;
    if (W < 1 || W > 64 || n_groups < 1 || n_groups > kMaxGroups || wp * n_groups > 64 || n_workers < 1 || n < 0 ||
        ring_cap == 0 || (ring_cap & (ring_cap - 1)))
        return -1;
    HostCtrl *ctrl = static_cast<HostCtrl *>(aligned_alloc(64, sizeof(HostCtrl)));
    memset((void *)ctrl, 0, sizeof(HostCtrl));
    DevDesc *ring = static_cast<DevDesc *>(aligned_alloc(256, sizeof(DevDesc) * ring_cap * n_groups));
    memset(ring, 0, sizeof(DevDesc) * ring_cap * n_groups);
    DevState *st = static_cast<DevState *>(aligned_alloc(256, sizeof(DevState)));
    memset(st, 0, sizeof(DevState));
    acs_trace_rec *tr = nullptr;
    if (trace_out && n > 0) {
        tr = static_cast<acs_trace_rec *>(calloc((size_t)n, sizeof(acs_trace_rec)));
    }
    DevParams p;
    memset(&p, 0, sizeof(p));
    p.ctrl = ctrl;
    p.ring = ring;
    p.st = st;
    p.trace = tr;
    p.ring_mask = ring_cap - 1;
    p.trace_cap = (uint32_t)n;
    p.W = W;
    p.n_workers = n_workers;
    p.n_groups = n_groups;
    p.host_check = host_check;
    p.check_wave = check_wave;

    const int nblk = 1 + n_workers;
    std::vector<std::unique_ptr<Block>> blocks;
    for (int b = 0; b < nblk; b++) {
        auto blk = std::make_unique<Block>();
        blk->bar = std::make_unique<std::barrier<>>(256);
        blk->g.bar = blk->bar.get();
        blocks.push_back(std::move(blk));
    }
    std::vector<std::thread> threads;
    for (int b = 0; b < nblk; b++)
        for (uint32_t t = 0; t < 256; t++) threads.emplace_back(run_thread, std::cref(p), blocks[b].get(), t, (uint32_t)b);

    const double t0 = now_s();
    int rc = 0;
    uint64_t sub[kMaxGroups] = {};
    for (int32_t i = 0; i < n && rc == 0; i++) {
        const int32_t g = groups ? groups[i] : 0;
        if (g < 0 || g >= n_groups) {
            rc = -1;
            break;
        }
        while (sub[g] - __atomic_load_n(&ctrl->consumed[g], __ATOMIC_SEQ_CST) >= ring_cap) {
            if (now_s() - t0 > timeout_s) {
                rc = -5;
                break;
            }
            std::this_thread::yield();
        }
        if (rc) break;
        DevDesc d;
        memset(&d, 0, sizeof(d));
        d.seq = (uint64_t)i;
        d.kid = descs[i].kid;
        d.npieces = descs[i].npieces;
        d.nseg = descs[i].nseg;
        d.wbits = descs[i].wbits;
        memcpy(d.s, descs[i].s, sizeof(d.s));
        memcpy(d.e, descs[i].e, sizeof(d.e));
        memcpy(d.args, descs[i].args, sizeof(d.args));
        d.gseq = (uint32_t)sub[g];
        d.group = (uint32_t)g;
        if (host_up) d.host_up = host_up[i];
        if (host_up_hi) d.host_up_hi = host_up_hi[i];
        ring[(size_t)g * ring_cap + (sub[g] & (ring_cap - 1))] = d;
        sub[g]++;
        __atomic_store_n(&ctrl->tail[g], sub[g], __ATOMIC_SEQ_CST);
    }
    auto retired_total = [&]() {
        uint64_t r = 0;
        for (int g = 0; g < n_groups; g++) r += __atomic_load_n(&ctrl->retired[g], __ATOMIC_SEQ_CST);
        return r;
    };
    while (rc == 0 && retired_total() < (uint64_t)n) {
        if (now_s() - t0 > timeout_s) rc = -5;
        std::this_thread::yield();
    }
    __atomic_store_n(&ctrl->stop, rc == 0 ? 1ull : 2ull, __ATOMIC_SEQ_CST);
    for (auto &t : threads) t.join();
    if (retired_out) *retired_out = retired_total();
    if (tr) {
        for (int32_t i = 0; i < n; i++) {
            acs_trace_rec r = tr[i];
            if (r.t_start == INT64_MAX || r.t_end == 0) {
                r.t_start = -1;
                r.t_end = -1;
            } else {
                r.t_start *= 10;
                r.t_end *= 10;
            }
            if (r.t_dispatch > 0) r.t_dispatch *= 10;
            if (r.t_retire > 0) r.t_retire *= 10;
            trace_out[i] = r;
        }
        free(tr);
    }
    free(st);
    free(ring);
    free(ctrl);
    return rc;
}

int sim_run_groups(int32_t W, int32_t n_groups, int32_t n_workers, int32_t n, const sim_desc *descs,
                   const int32_t *groups, uint32_t ring_cap, acs_trace_rec *trace_out, double timeout_s,
                   uint64_t *retired_out)
{
    return run_sim(W, n_groups, 0, 0, n_workers, n, descs, groups, nullptr, ring_cap, trace_out, timeout_s, retired_out);
}

int sim_run(int32_t W, int32_t n_workers, int32_t n, const sim_desc *descs, uint32_t ring_cap,
            acs_trace_rec *trace_out, double timeout_s, uint64_t *retired_out)
{
    return run_sim(W, 1, 0, 0, n_workers, n, descs, nullptr, nullptr, ring_cap, trace_out, timeout_s, retired_out);
}

// Host-check mode: host_up[i] is descriptor i's upstream list from the
// caller (bit d: descriptor i - 1 - d), checked against the M before it.
int sim_run_hostcheck(int32_t W, int32_t M, int32_t n_workers, int32_t n, const sim_desc *descs,
                      const uint64_t *host_up, uint32_t ring_cap, acs_trace_rec *trace_out, double timeout_s,
                      uint64_t *retired_out)
{
    if (M < 1 || M > 64 || !host_up) return -1;
    return run_sim(W, 1, M, 0, n_workers, n, descs, nullptr, host_up, ring_cap, trace_out, timeout_s, retired_out);
}

// The same with host lists longer than 64: host_up_hi[i] bit b is the kernel
// b + 65 places before kernel i.
int sim_run_hostcheck2(int32_t W, int32_t M, int32_t n_workers, int32_t n, const sim_desc *descs,
                       const uint64_t *host_up, const uint64_t *host_up_hi, uint32_t ring_cap, acs_trace_rec *trace_out,
                       double timeout_s, uint64_t *retired_out)
{
    if (M < 1 || M > ACS_HOST_CHECK_MAX || !host_up || !host_up_hi) return -1;
    return run_sim(W, 1, M, 0, n_workers, n, descs, nullptr, host_up, ring_cap, trace_out, timeout_s, retired_out,
                   host_up_hi);
}

// Check-wave mode: wave 2 computes each descriptor's upstream list over
// the 64 before it; the caller provides none.
int sim_run_checkwave(int32_t W, int32_t n_workers, int32_t n, const sim_desc *descs, uint32_t ring_cap,
                      acs_trace_rec *trace_out, double timeout_s, uint64_t *retired_out)
{
    return run_sim(W, 1, 64, 1, n_workers, n, descs, nullptr, nullptr, ring_cap, trace_out, timeout_s, retired_out);
}

}  // extern "C"
