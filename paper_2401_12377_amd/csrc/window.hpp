// Host-side scheduling window (steps a2, a3, a6), shared by the plain path
// and the manual path.
#pragma once
#include <stdint.h>

#include <deque>
#include <vector>

#include "internal.hpp"
#include "segtable.hpp"

namespace acs {

class HostWindow {
public:
    HostWindow(int32_t W, size_t fifo_cap, bool trace, size_t trace_cap);

    bool fifo_full() const { return fifo_.size() >= fifo_cap_; }
    bool fifo_empty() const { return fifo_.empty(); }
    void fifo_push(const Desc &d) { fifo_.push_back(d); }
    bool drained() const { return fifo_.empty() && valid_ == 0; }
    bool full() const { return valid_ == ((W_ >= 64) ? ~0ull : ((1ull << W_) - 1ull)); }
    int32_t waiting() const { return __builtin_popcountll(valid_ & ~exec_); }

    // a2 + a3: while a slot is free, moves the FIFO head into the lowest free
    // slot and computes its upstream mask against every occupied slot.
    int admit();

    // Ready slots (valid, not executing, no upstream left), oldest first.
    int ready_slots(int32_t *out, int32_t cap) const;
    // Slots not yet handed out (ready or pending), oldest first.
    int waiting_slots(int32_t *out, int32_t cap) const;
    // Slots this slot still waits for (in the window, not retired).
    uint64_t upstream(int32_t slot) const { return up_[slot]; }
    bool poisoned(int32_t slot) const { return (poison_ >> slot) & 1ull; }
    void mark_executing(int32_t slot);
    // a6: frees the slot and clears it from every upstream mask.  A non-zero
    // status marks the kernel failed: every kernel waiting on it, and every
    // later kernel that conflicts with it, is poisoned (never run).
    void retire(int32_t slot, int32_t status, int64_t t_start = -1, int64_t t_end = -1);

    const Desc &slot_desc(int32_t s) const { return slots_[s]; }
    int32_t slot_of(uint64_t seq) const;
    int scheduled_list(acs_entry *out, int32_t cap, int32_t *n) const;

    uint64_t valid() const { return valid_; }
    uint64_t executing() const { return exec_; }
    uint64_t overlap_tests() const { return tests_; }
    uint64_t poisoned_count() const { return n_poisoned_; }
    uint64_t retired() const { return n_retired_; }
    uint64_t dispatched() const { return n_dispatched_; }
    int32_t first_error() const { return first_error_; }

    const std::vector<acs_trace_rec> &trace() const { return trace_; }

private:
    int32_t W_;
    size_t fifo_cap_;
    std::deque<Desc> fifo_;
    Desc slots_[ACS_W_MAX];
    SegTable table_;                  // each slot's ranges by position, for the conflict tests
    uint64_t up_[ACS_W_MAX] = {};
    uint64_t valid_ = 0, exec_ = 0, poison_ = 0;
    uint64_t ev_ = 0, tests_ = 0, n_poisoned_ = 0, n_retired_ = 0, n_dispatched_ = 0;
    int32_t first_error_ = 0;
    std::vector<Desc> failed_;        // ranges of failed or poisoned kernels
    bool poison_all_ = false;         // too many failures to track: poison everything
    bool trace_on_;
    size_t trace_cap_;
    std::vector<acs_trace_rec> trace_;
};

}  // namespace acs
