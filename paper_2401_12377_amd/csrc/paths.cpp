// Manual, in-order and plain (host window + HIP stream pool) paths.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>

#include <chrono>
#include <thread>
#include <deque>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"
#include "window.hpp"

namespace acs {

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace {

int hip_fail(hipError_t e, const char *what)
{
    set_error(ACS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return ACS_EDEVICE;
}

// ---------------------------------------------------------------------------
// manual path: window only; the caller plays the executor
// ---------------------------------------------------------------------------
class ManualPath : public Path {
public:
    ManualPath(int32_t W, const acs_config &cfg)
        : win_(W, (size_t)cfg.queue_depth, cfg.trace != 0, (size_t)cfg.trace_capacity)
    {
    }
    int submit(const Desc &d) override
    {
        if (win_.fifo_full()) {
            win_.admit();
            if (win_.fifo_full()) {
                set_error(ACS_EAGAIN, "input FIFO full; complete kernels first");
                return ACS_EAGAIN;
            }
        }
        win_.fifo_push(d);
        pump();
        return ACS_OK;
    }
    int sync(uint64_t) override
    {
        pump();
        if (!win_.drained()) {
            set_error(ACS_ETIMEDOUT, "manual window still holds kernels");
            return ACS_ETIMEDOUT;
        }
        return win_.first_error() ? ACS_EKERNEL : ACS_OK;
    }
    int take_ready(uint64_t *seqs, int32_t cap, int32_t *n) override
    {
        pump();
        int32_t slots[ACS_W_MAX];
        const int32_t k = win_.ready_slots(slots, ACS_W_MAX);
        int32_t c = 0;
        for (int32_t q = 0; q < k && c < cap; q++) {
            win_.mark_executing(slots[q]);
            seqs[c++] = win_.slot_desc(slots[q]).seq;
        }
        if (n) *n = c;
        return ACS_OK;
    }
    int complete(uint64_t seq, int32_t status) override
    {
        const int32_t s = win_.slot_of(seq);
        if (s < 0 || !((win_.executing() >> s) & 1ull)) {
            set_error(ACS_EINVAL, "kernel is not executing");
            return ACS_EINVAL;
        }
        win_.retire(s, status);
        pump();
        return ACS_OK;
    }
    int scheduled_list(acs_entry *out, int32_t cap, int32_t *n) override { return win_.scheduled_list(out, cap, n); }
    int trace_read(acs_trace_rec *out, int64_t cap, int64_t *n) override
    {
        const auto &t = win_.trace();
        int64_t c = 0;
        for (; c < (int64_t)t.size() && c < cap; c++) out[c] = t[c];
        if (n) *n = c;
        return ACS_OK;
    }
    void stats(acs_stats &s) override
    {
        s.retired = win_.retired();
        s.dispatched = win_.dispatched();
        s.overlap_tests = win_.overlap_tests();
        s.poisoned = win_.poisoned_count();
    }

private:
    // poisoned kernels that become ready are retired without running
    void pump()
    {
        for (;;) {
            win_.admit();
            int32_t slots[ACS_W_MAX];
            const int32_t k = win_.ready_slots(slots, ACS_W_MAX);
            bool any = false;
            for (int32_t q = 0; q < k; q++)
                if (win_.poisoned(slots[q])) {
                    win_.mark_executing(slots[q]);
                    win_.retire(slots[q], 0);
                    any = true;
                }
            if (!any) break;
        }
    }
    HostWindow win_;
};

// ---------------------------------------------------------------------------
// in-order path: the single-stream baseline, no window
// ---------------------------------------------------------------------------
class InorderPath : public Path {
public:
    explicit InorderPath(const acs_config &cfg) : cfg_(cfg) {}
    ~InorderPath() override { shutdown(); }
    int start() override
    {
        hipError_t e = hipSetDevice(cfg_.device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        if (cfg_.trace) {
            e = hipEventCreate(&base_);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
            e = hipEventRecord(base_, stream_);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        }
        return ACS_OK;
    }
    int submit(const Desc &d) override
    {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool tr = cfg_.trace && d.seq < (uint64_t)cfg_.trace_capacity;
        if (tr) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            (void)hipEventRecord(e0, stream_);
        }
        hipError_t e = launch_task(d.kid, d.args, d.npieces, stream_);
        if (e != hipSuccess) {
            if (!err_) err_ = ACS_EDEVICE;
            return hip_fail(e, "kernel launch");
        }
        if (tr) {
            (void)hipEventRecord(e1, stream_);
            pending_.push_back({d.seq, d.kid, e0, e1});
        }
        submitted_++;
        return ACS_OK;
    }
    int sync(uint64_t timeout_ns) override
    {
        if (!stream_) return err_;
        const uint64_t t0 = now_ns();
        for (;;) {
            hipError_t q = hipStreamQuery(stream_);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) {
                err_ = ACS_EDEVICE;
                return hip_fail(q, "stream");
            }
            if (timeout_ns && now_ns() - t0 > timeout_ns) {
                set_error(ACS_ETIMEDOUT, "sync timed out");
                return ACS_ETIMEDOUT;
            }
            _mm_pause();
        }
        retired_ = submitted_;
        resolve_trace();
        return err_;
    }
    int poll() override
    {
        if (!stream_ || err_) return err_;
        const hipError_t q = hipStreamQuery(stream_);
        if (q != hipSuccess && q != hipErrorNotReady) {
            err_ = ACS_EDEVICE;
            return hip_fail(q, "stream");
        }
        return ACS_OK;
    }
    int scheduled_list(acs_entry *, int32_t, int32_t *n) override
    {
        if (n) *n = 0;
        return ACS_OK;
    }
    int trace_read(acs_trace_rec *out, int64_t cap, int64_t *n) override
    {
        int64_t c = 0;
        for (; c < (int64_t)trace_.size() && c < cap; c++) out[c] = trace_[c];
        if (n) *n = c;
        return ACS_OK;
    }
    int shutdown() override
    {
        if (stream_) {
            (void)hipStreamSynchronize(stream_);
            resolve_trace();
            (void)hipStreamDestroy(stream_);
            stream_ = nullptr;
        }
        if (base_) {
            (void)hipEventDestroy(base_);
            base_ = nullptr;
        }
        return ACS_OK;
    }
    void stats(acs_stats &s) override
    {
        s.retired = retired_;
        s.dispatched = submitted_;
    }

private:
    struct Pend {
        uint64_t seq;
        int32_t kid;
        hipEvent_t e0, e1;
    };
    void resolve_trace()
    {
        for (auto &p : pending_) {
            float a = 0, b = 0;
            (void)hipEventElapsedTime(&a, base_, p.e0);
            (void)hipEventElapsedTime(&b, base_, p.e1);
            if (trace_.size() <= p.seq) trace_.resize(p.seq + 1);
            acs_trace_rec &r = trace_[p.seq];
            r.seq = (int64_t)p.seq;
            r.slot = 0;
            r.kernel_id = p.kid;
            r.ev_insert = 3 * (int64_t)p.seq;
            r.ev_dispatch = 3 * (int64_t)p.seq + 1;
            r.ev_retire = 3 * (int64_t)p.seq + 2;
            r.valid_mask = 0;
            r.up_mask = 0;
            r.t_start = (int64_t)((double)a * 1e6);
            r.t_end = (int64_t)((double)b * 1e6);
            r.t_dispatch = -1;
            r.t_retire = -1;
            (void)hipEventDestroy(p.e0);
            (void)hipEventDestroy(p.e1);
        }
        pending_.clear();
    }
    acs_config cfg_;
    hipStream_t stream_ = nullptr;
    hipEvent_t base_ = nullptr;
    uint64_t submitted_ = 0, retired_ = 0;
    int err_ = ACS_OK;
    std::vector<Pend> pending_;
    std::vector<acs_trace_rec> trace_;
};

// ---------------------------------------------------------------------------
// plain path: host window feeding a pool of streams (the ACS-SW structure of
// Section IV-B).  A ready kernel goes to an idle stream, else to the stream
// with the shortest queue; a pending kernel whose upstream kernels are all
// executing in one stream goes into that stream at once (stream order keeps
// the edge).  The kernels a stream takes in one scheduling round go out as
// one launch (a multi-task kernel: they never depend on each other), which
// divides the host's launch cost; on submit, kernels are held back until
// eight wait or the window is full.  Completions are seen through events,
// recorded only when a completion is needed: when the window is full with
// kernels waiting in the FIFO, when some kernel could not be handed out, or
// on a drain.  An event after the last kernel of a stream marks every kernel
// before it (in trace mode every launch gets its own pair, for the
// execution intervals).
// ---------------------------------------------------------------------------
class PlainPath : public Path {
    static constexpr size_t kDepth = ACS_W_MAX;   // kernels per stream (no window holds more)
    static constexpr int32_t kBatch = 8;          // kernels held back on submit before a hand-out
    static constexpr int32_t kMaxStreams = 64;
    struct InFlight {
        int32_t slot;
        int32_t ev;    // event index marking the end of this kernel, or -1 (a later entry's covers it)
        int32_t beg;   // trace mode: event index before the kernel, else -1
    };

public:
    PlainPath(int32_t W, const acs_config &cfg)
        : cfg_(cfg), win_(W, (size_t)cfg.queue_depth, cfg.trace != 0, (size_t)cfg.trace_capacity)
    {
    }
    ~PlainPath() override { shutdown(); }
    int start() override
    {
        hipError_t e = hipSetDevice(cfg_.device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        const int S = cfg_.n_streams;
        streams_.assign(S, nullptr);
        q_.assign(S, {});
        for (int s = 0; s < S; s++)
            if ((e = hipStreamCreateWithFlags(&streams_[s], hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
        // enough events for every kernel in flight (two each with a trace)
        const unsigned flags = cfg_.trace ? hipEventDefault : hipEventDisableTiming;
        const size_t nev = 2 * (size_t)ACS_W_MAX + 2;   // at most two per kernel in flight
        events_.assign(nev, nullptr);
        ev_refs_.assign(nev, 0);
        for (size_t k = 0; k < nev; k++) {
            if ((e = hipEventCreateWithFlags(&events_[k], flags)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            free_ev_.push_back((int32_t)k);
        }
        if (cfg_.trace) {
            if ((e = hipEventCreate(&base_)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            if ((e = hipEventRecord(base_, streams_[0])) != hipSuccess) return hip_fail(e, "hipEventRecord");
            (void)hipEventSynchronize(base_);
        }
        for (int32_t k = 0; k < ACS_W_MAX; k++) stream_of_[k] = -1;
        started_ = true;
        return ACS_OK;
    }
    int submit(const Desc &d) override
    {
        while (win_.fifo_full()) {
            if (cfg_.nonblocking) {
                progress();
                if (win_.fifo_full()) {
                    set_error(ACS_EAGAIN, "input FIFO full");
                    return ACS_EAGAIN;
                }
                break;
            }
            progress();
            _mm_pause();
        }
        win_.fifo_push(d);
        progress(false, true);
        return ACS_OK;
    }
    int sync(uint64_t timeout_ns) override
    {
        const uint64_t t0 = now_ns();
        while (!win_.drained()) {
            progress(true);
            if (win_.drained()) break;
            if (timeout_ns && now_ns() - t0 > timeout_ns) {
                set_error(ACS_ETIMEDOUT, "sync timed out");
                return ACS_ETIMEDOUT;
            }
            _mm_pause();
        }
        if (dev_err_) return dev_err_;
        return win_.first_error() ? ACS_EKERNEL : ACS_OK;
    }
    int poll() override
    {
        if (!started_) return ACS_OK;
        progress(true);   // a caller that polls waits for completions
        if (dev_err_) return dev_err_;
        return win_.first_error() ? ACS_EKERNEL : ACS_OK;
    }
    int scheduled_list(acs_entry *out, int32_t cap, int32_t *n) override { return win_.scheduled_list(out, cap, n); }
    int trace_read(acs_trace_rec *out, int64_t cap, int64_t *n) override
    {
        const auto &t = win_.trace();
        int64_t c = 0;
        for (; c < (int64_t)t.size() && c < cap; c++) out[c] = t[c];
        if (n) *n = c;
        return ACS_OK;
    }
    int shutdown() override
    {
        if (!started_) return ACS_OK;
        sync(0);
        for (size_t s = 0; s < streams_.size(); s++)
            if (streams_[s]) (void)hipStreamDestroy(streams_[s]);
        for (hipEvent_t ev : events_)
            if (ev) (void)hipEventDestroy(ev);
        if (base_) (void)hipEventDestroy(base_);
        streams_.clear();
        events_.clear();
        free_ev_.clear();
        q_.clear();
        base_ = nullptr;
        started_ = false;
        return ACS_OK;
    }
    void stats(acs_stats &s) override
    {
        s.retired = win_.retired();
        s.dispatched = win_.dispatched();
        s.overlap_tests = win_.overlap_tests();
        s.poisoned = win_.poisoned_count();
        s.n_streams = (int32_t)streams_.size();
    }

private:
    int32_t take_event()
    {
        const int32_t k = free_ev_.back();
        free_ev_.pop_back();
        ev_refs_[(size_t)k] = 0;
        return k;
    }
    // an event may mark several kernels (a batch): freed with the last
    void drop_event(int32_t k)
    {
        if (k >= 0 && --ev_refs_[(size_t)k] <= 0) free_ev_.push_back(k);
    }

    // Retires the front kernels of stream s up to and including the first
    // one whose end event has fired; false when none has.
    bool retire_front(size_t s)
    {
        auto &q = q_[s];
        size_t upto = 0;
        hipError_t q_err = hipSuccess;
        bool fired = false;
        for (size_t k = 0; k < q.size(); k++) {
            if (q[k].ev < 0) continue;
            const hipError_t r = hipEventQuery(events_[(size_t)q[k].ev]);
            if (r == hipErrorNotReady) break;
            fired = true;
            q_err = r;
            upto = k + 1;
        }
        if (!fired) return false;
        for (size_t k = 0; k < upto; k++) {
            const InFlight f = q.front();
            q.pop_front();
            int64_t ta = -1, tb = -1;
            if (cfg_.trace && f.beg >= 0 && f.ev >= 0) {
                float a = 0, b = 0;
                (void)hipEventElapsedTime(&a, base_, events_[(size_t)f.beg]);
                (void)hipEventElapsedTime(&b, base_, events_[(size_t)f.ev]);
                ta = (int64_t)((double)a * 1e6);
                tb = (int64_t)((double)b * 1e6);
            }
            int32_t status = 0;
            if (q_err != hipSuccess) {
                status = ACS_EDEVICE;
                if (!dev_err_) dev_err_ = ACS_EDEVICE;
                hip_fail(q_err, "kernel");
            }
            drop_event(f.ev);
            drop_event(f.beg);
            stream_of_[f.slot] = -1;
            win_.retire(f.slot, status, ta, tb);
        }
        return true;
    }

    // Launches the kernels of `slots` (mutually independent, already marked
    // executing) into stream s: one task alone as its own kernel, several as
    // one multi-task launch.  A launch error retires them as failed.
    void launch_batch(const int32_t *slots, int32_t k, size_t s)
    {
        int32_t beg = -1;
        if (cfg_.trace) {
            beg = take_event();
            (void)hipEventRecord(events_[(size_t)beg], streams_[s]);
        }
        hipError_t e;
        if (k == 1) {
            const Desc &d = win_.slot_desc(slots[0]);
            e = launch_task(d.kid, d.args, d.npieces, streams_[s]);
        } else {
            MultiParams mp;
            mp.n = (uint32_t)k;
            mp.total = 0;
            for (int32_t i = 0; i < k; i++) {
                const Desc &d = win_.slot_desc(slots[i]);
                MultiTask &t = mp.t[i];
                t.kid = d.kid;
                t.np = d.npieces;
                t.first = mp.total;
                t.pad = 0;
                memcpy(t.args, d.args, ACS_ARGS_MAX);
                mp.total += d.npieces;
            }
            e = launch_multi(mp, streams_[s]);
        }
        if (e != hipSuccess) {
            hip_fail(e, "kernel launch");
            if (!dev_err_) dev_err_ = ACS_EDEVICE;
            if (beg >= 0) free_ev_.push_back(beg);
            for (int32_t i = 0; i < k; i++) {
                stream_of_[slots[i]] = -1;
                win_.retire(slots[i], ACS_EDEVICE);
            }
            return;
        }
        int32_t end = -1;
        if (cfg_.trace) {
            end = take_event();
            (void)hipEventRecord(events_[(size_t)end], streams_[s]);
        }
        for (int32_t i = 0; i < k; i++) {
            InFlight f{slots[i], -1, -1};
            if (cfg_.trace) {
                f.ev = end;
                f.beg = beg;
                ev_refs_[(size_t)end]++;
                ev_refs_[(size_t)beg]++;
            }
            stream_of_[slots[i]] = (int32_t)s;
            q_[s].push_back(f);
        }
    }

    // One pass of the window module and the scheduler module: retire what
    // finished, admit from the FIFO, hand out what can run.  Everything that
    // can run in a pass is mutually independent (a kernel whose upstream
    // kernel is still waiting is not among them), so each stream takes its
    // share as one launch.
    void progress(bool drain = false, bool lazy = false)
    {
        for (size_t s = 0; s < streams_.size(); s++)
            if (!q_[s].empty()) retire_front(s);
        win_.admit();
        // On submit, kernels are held back until a batch is worth a launch:
        // kBatch of them wait, or the window is full (a drain, a poll or any
        // other call hands out everything at once).
        if (lazy && !win_.full() && win_.waiting() < kBatch) return;
        bool blocked = false;   // some kernel could not be handed out
        // One walk in age order.  A kernel joins the open batch of the stream
        // that runs all its upstream kernels; if one of those is in that very
        // batch, the batch is launched first (stream order then keeps the
        // edge) and the kernel opens the next one.  Ready kernels share one
        // stream per walk.
        int32_t open[kMaxStreams][kMultiMax];
        int32_t nopen[kMaxStreams] = {};
        uint64_t inbatch[kMaxStreams] = {};
        const int32_t S = (int32_t)streams_.size();
        auto flush = [&](int32_t s) {
            if (nopen[s] == 0) return;
            launch_batch(open[s], nopen[s], (size_t)s);
            nopen[s] = 0;
            inbatch[s] = 0;
        };
        for (bool again = true; again;) {
            again = false;
            int32_t cand[ACS_W_MAX];
            const int32_t k = win_.waiting_slots(cand, ACS_W_MAX);
            int32_t ready_stream = -1;
            for (int32_t c = 0; c < k; c++) {
                const int32_t slot = cand[c];
                const uint64_t up = win_.upstream(slot);
                if (up == 0 && win_.poisoned(slot)) {
                    win_.mark_executing(slot);
                    win_.retire(slot, 0);
                    again = true;   // a retirement may free an admission
                    continue;
                }
                int32_t s = -1;
                if (up == 0) {
                    if (ready_stream < 0) ready_stream = pick_stream();
                    s = ready_stream;
                } else if (!win_.poisoned(slot) && (up & ~win_.executing()) == 0) {
                    // every upstream kernel runs or is about to: all in one stream?
                    const int32_t s0 = stream_of_[__builtin_ctzll(up)];
                    bool same = s0 >= 0;
                    for (uint64_t m = up; m && same; m &= m - 1) same = stream_of_[__builtin_ctzll(m)] == s0;
                    if (same) s = s0;
                }
                if (s < 0 || q_[(size_t)s].size() + (size_t)nopen[s] >= kDepth) {
                    blocked = true;
                    continue;
                }
                if ((up & inbatch[s]) != 0 || nopen[s] == kMultiMax) flush(s);
                open[s][nopen[s]++] = slot;
                inbatch[s] |= 1ull << slot;
                win_.mark_executing(slot);
                stream_of_[slot] = s;
            }
            for (int32_t s = 0; s < S; s++) flush(s);
            if (win_.admit() > 0) again = true;
        }
        // completions are needed: an end event behind each stream's last kernel
        const bool need = drain || blocked || (win_.full() && !win_.fifo_empty());
        if (need && !cfg_.trace)
            for (size_t s = 0; s < streams_.size(); s++) {
                if (q_[s].empty() || q_[s].back().ev >= 0) continue;
                InFlight &last = q_[s].back();
                last.ev = take_event();
                ev_refs_[(size_t)last.ev] = 1;
                (void)hipEventRecord(events_[(size_t)last.ev], streams_[s]);
            }
    }

    // an idle stream, else the least loaded one with room (-1 if none)
    int32_t pick_stream()
    {
        const int32_t S = (int32_t)streams_.size();
        int32_t best = -1;
        for (int32_t k = 0; k < S; k++) {
            const int32_t s = (rr_ + k) % S;
            const size_t len = q_[(size_t)s].size();
            if (len == 0) {
                best = s;
                break;
            }
            if (len < kDepth && (best < 0 || len < q_[(size_t)best].size())) best = s;
        }
        if (best >= 0) rr_ = (best + 1) % S;
        return best;
    }

    acs_config cfg_;
    HostWindow win_;
    std::vector<hipStream_t> streams_;
    std::vector<std::deque<InFlight>> q_;
    std::vector<hipEvent_t> events_;
    std::vector<int32_t> free_ev_;
    std::vector<int32_t> ev_refs_;   // kernels each event marks
    int32_t stream_of_[ACS_W_MAX];
    hipEvent_t base_ = nullptr;
    int32_t rr_ = 0;
    int dev_err_ = ACS_OK;
    bool started_ = false;
};

// ---------------------------------------------------------------------------
// events path: the multi-stream baseline.  Every kernel is launched when it
// is submitted, into one of S streams; a dependency on a kernel of another
// stream becomes a wait on that kernel's completion event.  Dependencies
// come from the same range test, against every kernel that may still be
// running: the last kHist kernels, where a kernel leaves that history only
// after its event has fired (seen by a query before each submit and on every
// poll; the host waits for the oldest when the history is full).
// ---------------------------------------------------------------------------
class EventsPath : public Path {
public:
    explicit EventsPath(const acs_config &cfg) : cfg_(cfg) {}
    ~EventsPath() override { shutdown(); }
    int start() override
    {
        hipError_t e = hipSetDevice(cfg_.device);
        if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
        streams_.assign((size_t)cfg_.n_streams, nullptr);
        for (auto &st : streams_)
            if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
        for (int32_t i = 0; i < kHist + 1; i++) {
            hipEvent_t ev;
            if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
            free_events_.push_back(ev);
        }
        started_ = true;
        return ACS_OK;
    }
    int submit(const Desc &d) override
    {
        if (err_) return err_;
        // kernels already complete leave the history first, so that they
        // cost neither range tests nor waits
        if (int rc = retire_fired(8)) return rc;
        if ((int32_t)hist_.size() == kHist)
            if (int rc = retire_oldest()) return rc;
        // newest conflicting kernel per stream: stream order covers the older ones
        int32_t dep_on[ACS_W_MAX];
        int64_t newest = -1;
        int32_t pick = -1;
        for (int32_t s = 0; s < (int32_t)streams_.size(); s++) dep_on[s] = -1;
        for (int32_t k = (int32_t)hist_.size() - 1; k >= 0; k--) {
            const Rec &o = hist_[(size_t)k];
            if (dep_on[o.stream] >= 0) continue;
            if (descs_conflict(o.d, d, &tests_)) {
                dep_on[o.stream] = k;
                if ((int64_t)o.d.seq > newest) {
                    newest = (int64_t)o.d.seq;
                    pick = o.stream;
                }
            }
        }
        // the stream of the newest upstream kernel, else the next stream in turn
        if (pick < 0) {
            pick = rr_;
            rr_ = (rr_ + 1) % (int32_t)streams_.size();
        }
        hipStream_t st = streams_[(size_t)pick];
        hipError_t e;
        for (int32_t s = 0; s < (int32_t)streams_.size(); s++) {
            if (s == pick || dep_on[s] < 0) continue;
            if ((e = hipStreamWaitEvent(st, hist_[(size_t)dep_on[s]].ev, 0)) != hipSuccess) return fail_dev(e, "hipStreamWaitEvent");
        }
        if ((e = launch_task(d.kid, d.args, d.npieces, st)) != hipSuccess) return fail_dev(e, "kernel launch");
        Rec r;
        r.d = d;
        r.stream = pick;
        r.ev = free_events_.back();
        free_events_.pop_back();
        if ((e = hipEventRecord(r.ev, st)) != hipSuccess) return fail_dev(e, "hipEventRecord");
        hist_.push_back(r);
        submitted_++;
        return ACS_OK;
    }
    int sync(uint64_t timeout_ns) override
    {
        const uint64_t t0 = now_ns();
        for (auto st : streams_) {
            for (;;) {
                const hipError_t q = hipStreamQuery(st);
                if (q == hipSuccess) break;
                if (q != hipErrorNotReady) return fail_dev(q, "stream");
                if (timeout_ns && now_ns() - t0 > timeout_ns) {
                    set_error(ACS_ETIMEDOUT, "sync timed out");
                    return ACS_ETIMEDOUT;
                }
                _mm_pause();
            }
        }
        while (!hist_.empty()) {
            free_events_.push_back(hist_.front().ev);
            hist_.erase(hist_.begin());
        }
        retired_ = submitted_;
        return err_;
    }
    int poll() override
    {
        if (err_) return err_;
        if (int rc = retire_fired(kHist)) return rc;
        return err_;
    }
    int scheduled_list(acs_entry *, int32_t, int32_t *n) override
    {
        if (n) *n = 0;
        return ACS_OK;
    }
    int trace_read(acs_trace_rec *, int64_t, int64_t *n) override
    {
        if (n) *n = 0;
        return ACS_OK;
    }
    int shutdown() override
    {
        if (!started_) return ACS_OK;
        (void)sync(0);
        for (auto st : streams_)
            if (st) (void)hipStreamDestroy(st);
        for (auto ev : free_events_) (void)hipEventDestroy(ev);
        streams_.clear();
        free_events_.clear();
        started_ = false;
        return ACS_OK;
    }
    void stats(acs_stats &s) override
    {
        s.retired = retired_;
        s.dispatched = submitted_;
        s.overlap_tests = tests_;
        s.n_streams = (int32_t)streams_.size();
    }

private:
    static constexpr int32_t kHist = 64;
    struct Rec {
        Desc d;
        int32_t stream = 0;
        hipEvent_t ev = nullptr;
    };
    // up to `max` kernels whose events have fired leave the history, oldest
    // first (a query per kernel, none waits)
    int retire_fired(int32_t max)
    {
        for (int32_t q = 0; q < max && !hist_.empty(); q++) {
            const hipError_t e = hipEventQuery(hist_.front().ev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return fail_dev(e, "hipEventQuery");
            free_events_.push_back(hist_.front().ev);
            hist_.erase(hist_.begin());
            retired_++;
        }
        return ACS_OK;
    }
    int retire_oldest()
    {
        const hipError_t e = hipEventSynchronize(hist_.front().ev);
        if (e != hipSuccess) return fail_dev(e, "hipEventSynchronize");
        free_events_.push_back(hist_.front().ev);
        hist_.erase(hist_.begin());
        retired_++;
        return ACS_OK;
    }
    int fail_dev(hipError_t e, const char *what)
    {
        if (!err_) err_ = ACS_EDEVICE;
        return hip_fail(e, what);
    }
    acs_config cfg_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> free_events_;
    std::vector<Rec> hist_;
    int32_t rr_ = 0;
    uint64_t submitted_ = 0, retired_ = 0, tests_ = 0;
    int err_ = ACS_OK;
    bool started_ = false;
};

}  // namespace

std::unique_ptr<Path> make_events_path(const acs_config &cfg) { return std::make_unique<EventsPath>(cfg); }
std::unique_ptr<Path> make_manual_path(int32_t W, const acs_config &cfg) { return std::make_unique<ManualPath>(W, cfg); }
std::unique_ptr<Path> make_inorder_path(const acs_config &cfg) { return std::make_unique<InorderPath>(cfg); }
std::unique_ptr<Path> make_plain_path(int32_t W, const acs_config &cfg) { return std::make_unique<PlainPath>(W, cfg); }

}  // namespace acs
