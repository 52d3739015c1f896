// Host-side scheduling window.
#include "window.hpp"

#include <algorithm>

namespace acs {

namespace {
constexpr size_t kMaxFailedTracked = 256;
}

HostWindow::HostWindow(int32_t W, size_t fifo_cap, bool trace, size_t trace_cap)
    : W_(W), fifo_cap_(fifo_cap), trace_on_(trace), trace_cap_(trace_cap)
{
}

int HostWindow::admit()
{
    const uint64_t full = (W_ >= 64) ? ~0ull : ((1ull << W_) - 1ull);
    int admitted = 0;
    while (!fifo_.empty() && valid_ != full) {
        const int32_t slot = __builtin_ctzll(~valid_);
        Desc &d = slots_[slot];
        d = fifo_.front();
        fifo_.pop_front();
        // every occupied slot at once (column = slot)
        tests_ += table_.pair_tests(valid_, d);
        const uint64_t up = table_.conflicts(valid_, d);
        table_.put(slot, d);
        bool bad = poison_all_;
        for (size_t k = 0; k < failed_.size() && !bad; k++) bad = descs_conflict(failed_[k], d, &tests_);
        if (trace_on_ && d.seq < trace_cap_) {
            if (trace_.size() <= d.seq) trace_.resize(d.seq + 1);
            acs_trace_rec &r = trace_[d.seq];
            r.seq = (int64_t)d.seq;
            r.slot = slot;
            r.kernel_id = d.kid;
            r.ev_insert = (int64_t)ev_;
            r.ev_dispatch = -1;
            r.ev_retire = -1;
            r.valid_mask = valid_;
            r.up_mask = up;
            r.t_start = -1;
            r.t_end = -1;
            r.t_dispatch = -1;
            r.t_retire = -1;
        }
        ev_++;
        up_[slot] = up;
        valid_ |= 1ull << slot;
        if (bad) poison_ |= 1ull << slot;
        admitted++;
    }
    return admitted;
}

int HostWindow::ready_slots(int32_t *out, int32_t cap) const
{
    int32_t n = 0;
    for (uint64_t m = valid_ & ~exec_; m; m &= m - 1) {
        const int32_t i = __builtin_ctzll(m);
        if (up_[i] == 0) out[n++] = i;
        if (n == cap) break;
    }
    std::sort(out, out + n, [this](int32_t a, int32_t b) { return slots_[a].seq < slots_[b].seq; });
    return n;
}

int HostWindow::waiting_slots(int32_t *out, int32_t cap) const
{
    int32_t n = 0;
    for (uint64_t m = valid_ & ~exec_; m && n < cap; m &= m - 1) out[n++] = __builtin_ctzll(m);
    std::sort(out, out + n, [this](int32_t a, int32_t b) { return slots_[a].seq < slots_[b].seq; });
    return n;
}

void HostWindow::mark_executing(int32_t slot)
{
    exec_ |= 1ull << slot;
    n_dispatched_++;
    const uint64_t seq = slots_[slot].seq;
    if (trace_on_ && seq < trace_.size()) trace_[seq].ev_dispatch = (int64_t)ev_;
    ev_++;
}

void HostWindow::retire(int32_t slot, int32_t status, int64_t t_start, int64_t t_end)
{
    const uint64_t bit = 1ull << slot;
    const Desc &d = slots_[slot];
    const bool failed = status != 0 || (poison_ & bit);
    if (failed) {
        if (status != 0 && first_error_ == 0) first_error_ = status;
        if (poison_ & bit) n_poisoned_++;
        // everything still waiting on this kernel inherits the failure
        for (uint64_t m = valid_; m; m &= m - 1) {
            const int32_t j = __builtin_ctzll(m);
            if (up_[j] & bit) poison_ |= 1ull << j;
        }
        if (failed_.size() < kMaxFailedTracked)
            failed_.push_back(d);
        else
            poison_all_ = true;
    }
    if (trace_on_ && d.seq < trace_.size()) {
        trace_[d.seq].ev_retire = (int64_t)ev_;
        trace_[d.seq].t_start = t_start;
        trace_[d.seq].t_end = t_end;
    }
    ev_++;
    for (int32_t j = 0; j < W_; j++) up_[j] &= ~bit;
    valid_ &= ~bit;
    exec_ &= ~bit;
    poison_ &= ~bit;
    n_retired_++;
}

int32_t HostWindow::slot_of(uint64_t seq) const
{
    for (uint64_t m = valid_; m; m &= m - 1) {
        const int32_t i = __builtin_ctzll(m);
        if (slots_[i].seq == seq) return i;
    }
    return -1;
}

int HostWindow::scheduled_list(acs_entry *out, int32_t cap, int32_t *n) const
{
    int32_t idx[ACS_W_MAX];
    int32_t k = 0;
    for (uint64_t m = valid_; m; m &= m - 1) idx[k++] = __builtin_ctzll(m);
    std::sort(idx, idx + k, [this](int32_t a, int32_t b) { return slots_[a].seq < slots_[b].seq; });
    int32_t c = 0;
    for (int32_t q = 0; q < k && c < cap; q++) {
        const int32_t i = idx[q];
        acs_entry &e = out[c++];
        e.seq = slots_[i].seq;
        e.kernel_id = slots_[i].kid;
        e.state = ((exec_ >> i) & 1ull) ? ACS_EXECUTING : (up_[i] == 0 ? ACS_READY : ACS_PENDING);
        e.upstream_mask = up_[i];
        e.slot = i;
        e.reserved = 0;
    }
    if (n) *n = c;
    return ACS_OK;
}

}  // namespace acs
