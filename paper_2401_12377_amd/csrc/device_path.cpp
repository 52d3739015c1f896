// Host side of the device-resident path: descriptor ring in pinned host
// memory, persistent kernel launch, completion counter polling.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dev_shared.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "segtable.hpp"

namespace acs {

namespace {

int hip_fail(hipError_t e, const char *what)
{
    set_error(ACS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return ACS_EDEVICE;
}

uint32_t pow2_at_least(uint32_t x)
{
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Windows configured without allocation keep their host control block and
// descriptor rings in one caller-provided block of pinned host memory: the
// control block first (kStaticCtrlBytes), the rings after it.
constexpr uint64_t kStaticCtrlBytes = 4096;
static_assert(sizeof(HostCtrl) <= kStaticCtrlBytes, "host control block must fit its reserved bytes");

// Devices with a window configured without allocation open (bit d): the
// static scheduler state of a device serves one such window at a time.
std::atomic<uint64_t> g_static_busy{0};

constexpr int32_t kStaticDevices = 64;

class DevicePath : public Path {
public:
    DevicePath(int32_t W, const acs_config &cfg) : W_(W), cfg_(cfg) {}
    // Without allocation: host control block and rings in `host` (pinned,
    // host_bytes long), scheduler state in the device's static state, the
    // persistent kernel on the caller's stream, no timing events.
    DevicePath(int32_t W, const acs_config &cfg, void *host, uint64_t host_bytes, hipStream_t stream)
        : W_(W), cfg_(cfg), static_(true), claimed_(true), host_(host), host_bytes_(host_bytes)
    {
        stream_ = stream;
    }
    ~DevicePath() override { shutdown(); }

    // The objects of windows configured without allocation live in static
    // storage, one per device (placement new); deleting one only ends its
    // lifetime.  Others come from the heap.
    static void *operator new(size_t n) { return ::operator new(n, std::align_val_t(alignof(DevicePath))); }
    static void *operator new(size_t, void *where) { return where; }
    static void operator delete(void *p);

    int start() override
    {
        hipError_t e = hipSetDevice(cfg_.device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        int cus = 0, rate_khz = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg_.device);
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, cfg_.device);
        clock_khz_ = rate_khz > 0 ? rate_khz : 100000;
        int32_t per_cu = 0;
        if ((e = persistent_blocks_per_cu(std::max(1, std::min(cfg_.n_groups, kMaxGroups)), &per_cu)) != hipSuccess)
            return hip_fail(e, "occupancy query");
        const int32_t capacity = std::max(1, per_cu) * std::max(1, cus);
        int32_t workers = cfg_.n_workers > 0 ? cfg_.n_workers : cus;
        workers = std::min(workers, capacity - 1);
        if (workers < 1) {
            set_error(ACS_EDEVICE, "persistent kernel does not fit on the device");
            return ACS_EDEVICE;
        }
        n_workers_ = workers;

        groups_ = std::max(1, std::min(cfg_.n_groups, kMaxGroups));
        ring_cap_ = pow2_at_least((uint32_t)std::max(16, cfg_.queue_depth));
        const size_t ring_bytes = sizeof(DevDesc) * ring_cap_ * (size_t)groups_;
        if (static_) {
            if (int rc = start_static(ring_bytes)) return rc;
        } else {
            if ((e = hipHostMalloc((void **)&ctrl_, sizeof(HostCtrl), hipHostMallocCoherent | hipHostMallocMapped)) !=
                hipSuccess)
                return hip_fail(e, "hipHostMalloc(ctrl)");
            memset((void *)ctrl_, 0, sizeof(HostCtrl));
            if ((e = hipHostMalloc((void **)&ring_, ring_bytes, hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
                return hip_fail(e, "hipHostMalloc(ring)");
            memset((void *)ring_, 0, ring_bytes);
            if ((e = hipMalloc((void **)&st_, sizeof(DevState))) != hipSuccess) return hip_fail(e, "hipMalloc(state)");
            if ((e = hipMemset(st_, 0, sizeof(DevState))) != hipSuccess) return hip_fail(e, "hipMemset(state)");
            if (cfg_.trace) {
                trace_cap_ = (uint32_t)cfg_.trace_capacity;
                if ((e = hipMalloc((void **)&dtrace_, sizeof(acs_trace_rec) * trace_cap_)) != hipSuccess)
                    return hip_fail(e, "hipMalloc(trace)");
                if ((e = hipMemset(dtrace_, 0, sizeof(acs_trace_rec) * trace_cap_)) != hipSuccess)
                    return hip_fail(e, "hipMemset(trace)");
            }
            if ((e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        }

        DevParams p;
        memset(&p, 0, sizeof(p));
        p.ctrl = ctrl_;
        p.ring = ring_;
        p.st = st_;
        p.trace = dtrace_;
        p.ring_mask = ring_cap_ - 1;
        p.trace_cap = trace_cap_;
        p.W = W_;
        p.n_workers = n_workers_;
        p.n_groups = groups_;
        hc_ = groups_ == 1 ? std::max(0, std::min(cfg_.host_check_depth, ACS_HOST_CHECK_MAX)) : 0;
        // one window: the checks run ahead of it, on the host when asked,
        // else in the check wave unless the window wave is asked to make them
        fc_ = groups_ == 1 && hc_ == 0 && cfg_.window_check == 0;
        p.host_check = fc_ ? ACS_W_MAX : hc_;
        p.check_wave = fc_ ? 1 : 0;
        hist_n_ = 0;
        hist_col_ = 0;
        held_ranges_ = held_writes_ = 0;
        memset(col_ranges_, 0, sizeof(col_ranges_));
        memset(col_writes_, 0, sizeof(col_writes_));
        if (!static_) {
            if ((e = hipEventCreate(&ev0_)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            if ((e = hipEventCreate(&ev1_)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            if ((e = hipEventRecord(ev0_, stream_)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        if ((e = launch_persistent(p, 1 + n_workers_, stream_)) != hipSuccess) return hip_fail(e, "persistent kernel launch");
        if (!static_ && (e = hipEventRecord(ev1_, stream_)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        running_ = true;
        return ACS_OK;
    }

    // Start of a window configured without allocation (its object holds the
    // device's claim): checks the caller's memory and stream, and clears the
    // device's static state on the stream ahead of the persistent kernel.
    int start_static(size_t ring_bytes)
    {
        if (cfg_.trace) {
            set_error(ACS_EINVAL, "a window configured without allocation keeps no trace (set trace to 0)");
            return ACS_EINVAL;
        }
        const uint64_t need = kStaticCtrlBytes + ring_bytes;
        if (host_bytes_ < need) {
            set_error(ACS_EINVAL, "host block of " + std::to_string(host_bytes_) + " bytes; this configuration needs " +
                                      std::to_string(need));
            return ACS_EINVAL;
        }
        hipDevice_t sd = -1;
        hipError_t e = hipStreamGetDevice(stream_, &sd);
        if (e != hipSuccess) return hip_fail(e, "hipStreamGetDevice");
        if (sd != cfg_.device) {
            set_error(ACS_EINVAL, "the stream belongs to another device than the window");
            return ACS_EINVAL;
        }
        ctrl_ = static_cast<HostCtrl *>(host_);
        ring_ = reinterpret_cast<DevDesc *>(static_cast<uint8_t *>(host_) + kStaticCtrlBytes);
        memset((void *)ctrl_, 0, sizeof(HostCtrl));
        memset((void *)ring_, 0, ring_bytes);
        if ((e = static_state(cfg_.device, &st_)) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(state)");
        // the previous window's queue entries, counters and rings are still there
        if ((e = clear_state(st_, stream_)) != hipSuccess) return hip_fail(e, "clearing the scheduler state");
        return ACS_OK;
    }

    int submit(const Desc &d) override { return submit_group(d, 0); }

    int submit_group(const Desc &d, int32_t g) override
    {
        if (!running_) {
            set_error(ACS_ESTATE, "device path is not running");
            return ACS_ESTATE;
        }
        // back-pressure: each group's ring holds at most ring_cap_ unconsumed
        // descriptors.  The device-written counter is read only when the
        // cached value says the ring may be full (reading a line the device
        // keeps writing costs a cross-fabric miss).
        while (submitted_[g] - consumed_seen_[g] >= ring_cap_) {
            consumed_seen_[g] = __atomic_load_n(&ctrl_->consumed[g], __ATOMIC_ACQUIRE);
            if (submitted_[g] - consumed_seen_[g] < ring_cap_) break;
            if (cfg_.nonblocking) {
                set_error(ACS_EAGAIN, "input FIFO full");
                return ACS_EAGAIN;
            }
            if (int rc = check_alive()) return rc;
            _mm_pause();
        }
        DevDesc &r = ring_[(size_t)g * ring_cap_ + (submitted_[g] & (ring_cap_ - 1))];
        // Written in place (the ring is ordinary cached host memory, and the
        // device reads it only after the tail below says so).  With the
        // checks on the host the device reads only the head, so the ranges
        // are not written.
        r.seq = d.seq;
        r.kid = d.kid;
        r.npieces = d.npieces;
        r.gseq = (uint32_t)submitted_[g];   // the group's own numbering, without gaps
        r.group = (uint32_t)g;
        uint64_t up_lo = 0, up_hi = 0;
        if (hc_ > 0) host_check(d, up_lo, up_hi);
        r.host_up = up_lo;
        r.host_up_hi = up_hi;
        memcpy(r.args, d.args, ACS_ARGS_MAX);
        r.nseg = d.nseg;
        r.wbits = d.wbits;
        if (hc_ == 0) {
            memset(r.pad, 0, sizeof(r.pad));
            for (int k = 0; k < ACS_K_MAX; k++) {
                r.s[k] = d.s[k];
                r.e[k] = d.e[k];
            }
        }
        submitted_[g]++;
        total_submitted_++;
        __atomic_store_n(&ctrl_->tail[g], submitted_[g], __ATOMIC_RELEASE);
        return ACS_OK;
    }

    int sync(uint64_t timeout_ns) override
    {
        for (int32_t g = 0; g < groups_; g++)
            if (int rc = sync_group(g, timeout_ns)) return rc;
        return err_;
    }

    int sync_group(int32_t g, uint64_t timeout_ns) override
    {
        if (!running_) return err_;
        const uint64_t t0 = now_ns();
        uint32_t spins = 0;
        while (__atomic_load_n(&ctrl_->retired[g], __ATOMIC_ACQUIRE) < submitted_[g]) {
            if (++spins % 4096 == 0) {
                if (int rc = check_alive()) return rc;
                if (timeout_ns && now_ns() - t0 > timeout_ns) {
                    set_error(ACS_ETIMEDOUT, "sync timed out");
                    return ACS_ETIMEDOUT;
                }
            }
            _mm_pause();
        }
        if (ctrl_->error) err_ = ACS_EKERNEL;
        return err_;
    }

    int poll() override
    {
        if (!running_) return err_;
        if (++polls_ % 1024 == 0)
            if (int rc = check_alive()) return rc;
        if (ctrl_->error) err_ = ACS_EKERNEL;
        return err_;
    }

    int scheduled_list(acs_entry *out, int32_t cap, int32_t *n) override
    {
        if (!running_) {
            if (n) *n = 0;
            return ACS_OK;
        }
        const uint64_t req = ++snap_req_;
        __atomic_store_n(&ctrl_->snap_req, req, __ATOMIC_RELEASE);
        const uint64_t t0 = now_ns();
        while (__atomic_load_n(&ctrl_->snap_ack, __ATOMIC_ACQUIRE) < req) {
            if (now_ns() - t0 > 2000000000ull) {
                set_error(ACS_ETIMEDOUT, "no window snapshot from the device");
                return ACS_ETIMEDOUT;
            }
            std::this_thread::yield();
        }
        const int32_t cnt = (int32_t)std::min<uint64_t>((uint64_t)ctrl_->snap_count, (uint64_t)ACS_W_MAX);
        int32_t c = 0;
        for (; c < cnt && c < cap; c++) out[c] = ctrl_->snap[c];
        if (n) *n = c;
        return ACS_OK;
    }

    int trace_read(acs_trace_rec *out, int64_t cap, int64_t *n) override
    {
        if (!dtrace_) {
            if (n) *n = 0;
            return ACS_OK;
        }
        const int64_t cnt = (int64_t)std::min<uint64_t>(total_submitted_, trace_cap_);
        const int64_t c = std::min(cnt, cap);
        std::vector<acs_trace_rec> tmp((size_t)c);
        hipError_t e = hipMemcpy(tmp.data(), dtrace_, sizeof(acs_trace_rec) * (size_t)c, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(trace)");
        const double ns_per_tick = 1e6 / (double)clock_khz_;
        for (int64_t i = 0; i < c; i++) {
            acs_trace_rec r = tmp[(size_t)i];
            if (r.t_start == INT64_MAX || r.t_end == 0) {
                r.t_start = -1;
                r.t_end = -1;
            } else {
                r.t_start = (int64_t)((double)r.t_start * ns_per_tick);
                r.t_end = (int64_t)((double)r.t_end * ns_per_tick);
            }
            if (r.t_dispatch > 0) r.t_dispatch = (int64_t)((double)r.t_dispatch * ns_per_tick);
            if (r.t_retire > 0) r.t_retire = (int64_t)((double)r.t_retire * ns_per_tick);
            out[i] = r;
        }
        if (n) *n = c;
        return ACS_OK;
    }

    int stop() override
    {
        int rc = ACS_OK;
        if (running_) {
            rc = sync(10ull * 1000000000ull);
            __atomic_store_n(&ctrl_->stop, rc == ACS_OK ? 1ull : 2ull, __ATOMIC_RELEASE);
            if (!wait_exit(10ull * 1000000000ull)) {
                __atomic_store_n(&ctrl_->stop, 2ull, __ATOMIC_RELEASE);
                if (!wait_exit(10ull * 1000000000ull)) {
                    // the kernel did not leave: keep its memory rather than free it under a running kernel
                    set_error(ACS_EDEVICE, "persistent kernel did not exit");
                    running_ = false;
                    leaked_ = true;
                    return ACS_EDEVICE;
                }
            }
            checks_ = ctrl_->checks + ctrl_->check_wave_tests[0] + ctrl_->check_wave_tests[1];
            running_ = false;
            // Workers take tickets with one wave-wide add of 1 per lane, which
            // counts kWave per ticket only if the adds were combined into one
            // read-modify-write; every worker takes one exit ticket.  Check
            // that the count came out exactly so after a clean exit.
            if (rc == ACS_OK && ctrl_->exited) {
                uint64_t deq = 0;
                const hipError_t e = hipMemcpy(&deq, &st_->deq, sizeof(deq), hipMemcpyDeviceToHost);
                if (e != hipSuccess) {
                    rc = hip_fail(e, "hipMemcpy(queue head)");
                } else if (deq != 64ull * (ctrl_->published + (uint64_t)n_workers_)) {
                    set_error(ACS_EDEVICE, "work-queue tickets do not add up: the workers' ticket count is broken");
                    rc = ACS_EDEVICE;
                }
                if (rc != ACS_OK && err_ == ACS_OK) err_ = rc;
            }
            float ms = 0.0f;
            if (ev0_ && hipEventElapsedTime(&ms, ev0_, ev1_) == hipSuccess) kernel_ns_ = (uint64_t)((double)ms * 1e6);
        }
        return rc;
    }

    int shutdown() override
    {
        const int rc = stop();
        if (leaked_) return rc;
        if (static_) {
            // the caller's memory and stream stay the caller's
            if (claimed_) g_static_busy.fetch_and(~(1ull << cfg_.device), std::memory_order_acq_rel);
            claimed_ = false;
            st_ = nullptr;
            ring_ = nullptr;
            ctrl_ = nullptr;
            stream_ = nullptr;
            return rc;
        }
        if (stream_) {
            (void)hipStreamDestroy(stream_);
            stream_ = nullptr;
        }
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        ev0_ = ev1_ = nullptr;
        if (st_) (void)hipFree(st_);
        if (dtrace_) (void)hipFree(dtrace_);
        if (ring_) (void)hipHostFree((void *)ring_);
        if (ctrl_) (void)hipHostFree((void *)ctrl_);
        st_ = nullptr;
        dtrace_ = nullptr;
        ring_ = nullptr;
        ctrl_ = nullptr;
        return rc;
    }

    void stats(acs_stats &s) override
    {
        uint64_t ret = 0;
        for (int32_t g = 0; g < groups_; g++) ret += ctrl_ ? ctrl_->retired[g] : submitted_[g];
        s.retired = ret;
        s.dispatched = s.retired;
        s.overlap_tests = (running_ && ctrl_ ? ctrl_->checks + ctrl_->check_wave_tests[0] + ctrl_->check_wave_tests[1]
                                            : checks_) +
                          host_tests_;
        s.n_workers = n_workers_;
        s.kernel_ns = kernel_ns_;
    }

private:
    // Host-check mode (the split of Section IV-C): the new kernel is checked
    // against the M kernels submitted before it (one window group, numbered
    // without gaps), the host's scheduled list.  The list is stale by design:
    // some of them may have completed (the workers find those complete), and
    // none older can still be in the window when the kernel is inserted (the
    // device holds it back until that is so).  Bit b of lo: the kernel b + 1
    // places back; bit b of hi: the kernel b + 65 places back (M > 64).
    void host_check(const Desc &d, uint64_t &lo, uint64_t &hi)
    {
        const int32_t M = hc_;
        // Kernel j of the list sits in column j mod M (columns 64 and up in
        // the second table), and hist_col_ is the column of the next one: the
        // list fills columns 0 .. n - 1 (all M once it is full), and column c
        // holds the kernel (hist_col_ - 1 - c) mod M + 1 places back.
        const uint64_t n = std::min<uint64_t>((uint64_t)M, hist_n_);
        // segment pairs the definition compares: a write against every held
        // range, a read against every held write (running totals of the list)
        const uint32_t nw = (uint32_t)__builtin_popcount(d.wbits & ((1u << d.nseg) - 1u));
        host_tests_ += (uint64_t)nw * held_ranges_ + (uint64_t)(d.nseg - nw) * held_writes_;
        lo = hi = 0;
        for (int32_t t = 0; t < 2 && 64ull * (uint64_t)t < n; t++) {
            const uint64_t cnt = n - 64ull * (uint64_t)t;
            const uint64_t cols = cnt >= 64 ? ~0ull : (1ull << cnt) - 1ull;
            for (uint64_t hit = hist_[t].conflicts(cols, d); hit; hit &= hit - 1) {
                int32_t b = hist_col_ - 1 - (64 * t + __builtin_ctzll(hit));
                b += b < 0 ? M : 0;
                if (b < 64)
                    lo |= 1ull << b;
                else
                    hi |= 1ull << (b - 64);
            }
        }
        held_ranges_ += d.nseg - col_ranges_[hist_col_];
        held_writes_ += nw - col_writes_[hist_col_];
        col_ranges_[hist_col_] = (uint8_t)d.nseg;
        col_writes_[hist_col_] = (uint8_t)nw;
        hist_[hist_col_ / 64].put(hist_col_ % 64, d);
        hist_col_ = hist_col_ + 1 == M ? 0 : hist_col_ + 1;
        hist_n_++;
    }

    // A persistent kernel that left early (fault or abort) can no longer
    // retire anything: report it instead of spinning forever.
    int check_alive()
    {
        const hipError_t q = hipStreamQuery(stream_);
        if (q == hipErrorNotReady) return ACS_OK;
        running_ = false;
        err_ = ACS_EDEVICE;
        if (q != hipSuccess) return hip_fail(q, "persistent kernel");
        set_error(ACS_EDEVICE, "persistent kernel exited");
        return ACS_EDEVICE;
    }
    bool wait_exit(uint64_t timeout_ns)
    {
        const uint64_t t0 = now_ns();
        for (;;) {
            const hipError_t q = hipStreamQuery(stream_);
            if (q != hipErrorNotReady) return true;
            if (now_ns() - t0 > timeout_ns) return false;
            std::this_thread::yield();
        }
    }

    int32_t W_;
    uint64_t polls_ = 0;
    int32_t hc_ = 0;                 // host-check depth M (0: checks on the device)
    bool fc_ = false;                // checks made by the check wave
    SegTable hist_[2];               // the last M kernels submitted, kernel j in column j % M
                                     // (columns 64 and up in the second table)
    uint64_t hist_n_ = 0;
    int32_t hist_col_ = 0;           // column of the next kernel: hist_n_ mod M
    uint8_t col_ranges_[ACS_HOST_CHECK_MAX] = {}, col_writes_[ACS_HOST_CHECK_MAX] = {};   // ranges and writes
                                                                                          // of each column's kernel
    uint32_t held_ranges_ = 0, held_writes_ = 0;        // their sums over the list
    uint64_t host_tests_ = 0;
    acs_config cfg_;
    HostCtrl *ctrl_ = nullptr;
    DevDesc *ring_ = nullptr;
    DevState *st_ = nullptr;
    acs_trace_rec *dtrace_ = nullptr;
    hipStream_t stream_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    uint64_t kernel_ns_ = 0;
    uint32_t ring_cap_ = 0, trace_cap_ = 0;
    int32_t n_workers_ = 0;
    int clock_khz_ = 100000;
    int32_t groups_ = 1;
    uint64_t submitted_[kMaxGroups] = {}, consumed_seen_[kMaxGroups] = {};
    uint64_t total_submitted_ = 0, snap_req_ = 0, checks_ = 0;
    int err_ = ACS_OK;
    bool running_ = false, leaked_ = false;
    bool static_ = false, claimed_ = false;
    void *host_ = nullptr;
    uint64_t host_bytes_ = 0;
};

alignas(DevicePath) uint8_t g_static_paths[kStaticDevices][sizeof(DevicePath)];

void DevicePath::operator delete(void *p)
{
    const uint8_t *b = static_cast<const uint8_t *>(p);
    const uint8_t *lo = &g_static_paths[0][0];
    if (b >= lo && b < lo + sizeof(g_static_paths)) return;
    ::operator delete(p, std::align_val_t(alignof(DevicePath)));
}

}  // namespace

std::unique_ptr<Path> make_device_path(int32_t W, const acs_config &cfg) { return std::make_unique<DevicePath>(W, cfg); }

std::unique_ptr<Path> make_device_path_static(int32_t W, const acs_config &cfg, void *host, uint64_t host_bytes,
                                              void *stream, int *rc)
{
    if (cfg.device < 0 || cfg.device >= kStaticDevices) {
        set_error(ACS_EINVAL, "windows without allocation serve devices 0 to 63");
        *rc = ACS_EINVAL;
        return nullptr;
    }
    // One object slot and one scheduler state per device: the claim taken
    // here is released when the object is destroyed.
    const uint64_t bit = 1ull << cfg.device;
    if (g_static_busy.fetch_or(bit, std::memory_order_acq_rel) & bit) {
        set_error(ACS_ESTATE, "a window configured without allocation is already open on this device");
        *rc = ACS_ESTATE;
        return nullptr;
    }
    *rc = ACS_OK;
    return std::unique_ptr<Path>(new (static_cast<void *>(g_static_paths[cfg.device]))
                                     DevicePath(W, cfg, host, host_bytes, static_cast<hipStream_t>(stream)));
}

}  // namespace acs
