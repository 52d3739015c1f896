// Serving loop and its working-memory pool (acs_workloads.h): requests
// arrive over time, are admitted by working-memory footprint and request
// slots, and run concurrently through one open window.  Completion reaches
// the host through signal kernels that the window orders after the request's
// kernels, so the loop never drains the window while it runs.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>

#include <chrono>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "acs.h"
#include "acs_tasks.h"
#include "acs_workloads.h"
#include "drivers.hpp"
#include "internal.hpp"
#include "rl_layout.hpp"

// Best fit over a free map keyed by offset; live blocks are remembered so
// that a free names only its address.
struct acs_pool {
    uint64_t base = 0, bytes = 0, used = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> size
    std::map<uint64_t, uint64_t> live_;   // offset -> size

    bool alloc(uint64_t want, uint64_t *addr)
    {
        const uint64_t sz = acs::rl_align(want);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= sz && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return false;
        const uint64_t off = best->first, have = best->second;
        free_.erase(best);
        if (have > sz) free_[off + sz] = have - sz;
        live_[off] = sz;
        used += sz;
        *addr = base + off;
        return true;
    }

    bool release(uint64_t addr)
    {
        if (addr < base) return false;
        auto it = live_.find(addr - base);
        if (it == live_.end()) return false;
        uint64_t off = it->first, sz = it->second;
        live_.erase(it);
        used -= sz;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + sz == next->first) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += sz;
                return true;
            }
        }
        free_[off] = sz;
        return true;
    }

    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &f : free_) m = f.second > m ? f.second : m;
        return m;
    }
};

extern "C" {

acs_pool *acs_pool_create(uint64_t base, uint64_t bytes)
{
    if (base % 256 != 0 || bytes < 256 || bytes > UINT64_MAX - base) return nullptr;
    acs_pool *p = new (std::nothrow) acs_pool;
    if (!p) return nullptr;
    p->base = base;
    p->bytes = bytes & ~uint64_t(255);
    p->free_[0] = p->bytes;
    return p;
}

int acs_pool_alloc(acs_pool *p, uint64_t bytes, uint64_t *addr)
{
    if (!p || !addr || bytes == 0 || bytes > p->bytes) return bytes > 0 && p && addr ? ACS_ENOMEM : ACS_EINVAL;
    return p->alloc(bytes, addr) ? ACS_OK : ACS_ENOMEM;
}

int acs_pool_free(acs_pool *p, uint64_t addr)
{
    if (!p) return ACS_EINVAL;
    return p->release(addr) ? ACS_OK : ACS_EINVAL;
}

int acs_pool_info(const acs_pool *p, uint64_t *used, uint64_t *largest_free, int64_t *n_blocks)
{
    if (!p) return ACS_EINVAL;
    if (used) *used = p->used;
    if (largest_free) *largest_free = p->largest_free();
    if (n_blocks) *n_blocks = (int64_t)p->live_.size();
    return ACS_OK;
}

void acs_pool_destroy(acs_pool *p) { delete p; }

}  // extern "C"

namespace {

double clock_ns()
{
    return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t kPlanSlotBytes = 4 * 4 * (1 + acs::kRLMaxBodies / 2 + 1);   // >= rl_plan_ints(1024) ints

uint64_t host_bytes(int32_t R) { return acs::rl_align(8 * (uint64_t)R) + kPlanSlotBytes * (uint64_t)R; }

// Tokens the signal kernels store: unique per (request, phase).
uint64_t token(int32_t req, int32_t phase) { return ((uint64_t)(req + 1) << 2) | (uint64_t)phase; }

struct Slot {
    int32_t req = -1;
    int32_t phase = 0;           // 1: waiting for the plan, 2: waiting for the final signal
    int32_t group = 0;
    uint64_t block = 0, bytes = 0;
    acs_rl_scene scene = {};
    std::unique_ptr<acs::RLStep> rl;
    acs_rl_counts counts = {};
};

class Server {
public:
    Server(acs_window *w, const acs_serve_config &cfg, const acs_serve_request *req, int32_t n,
           acs_serve_result *res)
        : w_(w), cfg_(cfg), req_(req), n_(n), res_(res)
    {
    }
    ~Server()
    {
        if (pool_) acs_pool_destroy(pool_);
    }

    int validate()
    {
        if (cfg_.max_resident < 1 || cfg_.max_resident > 1024) return ACS_EINVAL;
        if (!cfg_.host || (uintptr_t)cfg_.host % 256 != 0 || cfg_.host_bytes < host_bytes(cfg_.max_resident))
            return ACS_EINVAL;
        groups_ = w_->configured ? w_->cfg.n_groups : 1;
        for (int32_t i = 0; i < n_; i++) {
            const acs_serve_request &q = req_[i];
            if (i > 0 && q.arrival_ns < req_[i - 1].arrival_ns) return ACS_EINVAL;
            if (q.kind == ACS_SERVE_RL) {
                if (q.n < 2 || q.n > acs::kRLMaxBodies || q.iters < 0 || q.iters % 2 != 0 || !q.input || !q.output)
                    return ACS_EINVAL;
            } else if (q.kind == ACS_SERVE_DNN) {
                if (!cfg_.model || !q.input || !q.output || !q.logits) return ACS_EINVAL;
            } else {
                return ACS_EINVAL;
            }
            if (footprint(q) > (cfg_.pool_bytes & ~uint64_t(255))) return ACS_EINVAL;
        }
        if (cfg_.model && (cfg_.model->n_cells < 1 || cfg_.model->n_cells > ACS_DNN_MAX_CELLS)) return ACS_EINVAL;
        return ACS_OK;
    }

    int setup()
    {
        pool_ = acs_pool_create(cfg_.pool, cfg_.pool_bytes);
        if (!pool_) return ACS_EINVAL;
        const int32_t R = cfg_.max_resident;
        flags_ = static_cast<uint64_t *>(cfg_.host);
        plans_ = static_cast<uint8_t *>(cfg_.host) + acs::rl_align(8 * (uint64_t)R);
        for (int32_t s = 0; s < R; s++) __atomic_store_n(&flags_[s], 0, __ATOMIC_RELEASE);
        slots_.resize((size_t)R);
        for (int32_t s = R - 1; s >= 0; s--) free_slots_.push_back(s);
        load_.assign((size_t)groups_, 0);
        return ACS_OK;
    }

    int run(acs_serve_stats *stats)
    {
        const uint64_t stall = cfg_.stall_ns ? cfg_.stall_ns : 60ull * 1000 * 1000 * 1000;
        const double t0 = clock_ns();
        int32_t arrived = 0, admitted = 0, done = 0;
        bool head_waited_mem = false, head_waited_slot = false;
        double last_progress = t0;
        while (done < n_) {
            const double now = clock_ns() - t0;
            while (arrived < n_ && req_[arrived].arrival_ns <= now) arrived++;
            // admission: the queue head only, in arrival order
            while (admitted < arrived) {
                if (free_slots_.empty()) {
                    if (!head_waited_slot) stats_.waited_resident++;
                    head_waited_slot = true;
                    break;
                }
                uint64_t block = 0;
                const uint64_t need = footprint(req_[admitted]);
                if (acs_pool_alloc(pool_, need, &block) != ACS_OK) {
                    if (!head_waited_mem) stats_.waited_memory++;
                    head_waited_mem = true;
                    break;
                }
                head_waited_mem = head_waited_slot = false;
                if (int rc = admit(admitted, block, need, clock_ns() - t0)) return rc;
                admitted++;
                last_progress = clock_ns();
            }
            // completions and plan signals
            for (size_t k = 0; k < resident_.size();) {
                const int32_t s = resident_[k];
                Slot &sl = slots_[(size_t)s];
                const uint64_t v = __atomic_load_n(&flags_[s], __ATOMIC_ACQUIRE);
                if (v != token(sl.req, sl.phase)) {
                    k++;
                    continue;
                }
                if (sl.phase == 1 && !sl.rl->plan_ready()) {
                    k++;   // signalled, but the plan's stamp has not reached host memory yet
                    continue;
                }
                last_progress = clock_ns();
                if (sl.phase == 1) {
                    if (int rc = submit_rl_tail(s)) return rc;
                    k++;
                    continue;
                }
                if (res_) res_[sl.req].done_ns = clock_ns() - t0;
                if (acs_pool_free(pool_, sl.block) != ACS_OK) return ACS_EINVAL;
                load_[(size_t)sl.group]--;
                sl.rl.reset();
                sl.req = -1;
                free_slots_.push_back(s);
                resident_[k] = resident_.back();
                resident_.pop_back();
                done++;
            }
            if (int rc = acs_poll(w_)) return rc;
            if (!resident_.empty() && clock_ns() - last_progress > (double)stall) {
                acs::set_error(ACS_ETIMEDOUT, "serving: no request made progress");
                return ACS_ETIMEDOUT;
            }
            if (resident_.empty() && admitted == arrived) last_progress = clock_ns();
            _mm_pause();
        }
        const int rc = acs_sync(w_);
        stats_.wall_ns = clock_ns() - t0;
        if (stats) *stats = stats_;
        return rc;
    }

private:
    uint64_t footprint(const acs_serve_request &q) const
    {
        if (q.kind == ACS_SERVE_RL) {
            uint64_t off[ACS_RL_NREGIONS];
            acs::rl_offsets(q.n, off);
            return off[ACS_RL_END];
        }
        return acs::dnn_activation_bytes(cfg_.model);
    }

    int32_t pick_group() const
    {
        int32_t g = 0;
        for (int32_t k = 1; k < groups_; k++)
            if (load_[(size_t)k] < load_[(size_t)g]) g = k;
        return g;
    }

    int submit(Slot &sl, int32_t kid, const acs_seg *r, int32_t nr, const acs_seg *wr, int32_t nw, const void *a,
               size_t asz)
    {
        const int rc = acs_submit_group(w_, sl.group, kid, r, nr, wr, nw, a, asz, nullptr);
        if (rc == ACS_OK) count(sl, 1);
        return rc;
    }

    void count(Slot &sl, uint64_t k)
    {
        stats_.kernels += k;
        if (res_) res_[sl.req].kernels += k;
    }

    int signal(Slot &sl, int32_t s, const acs_seg *r, int32_t nr)
    {
        const acs_args_signal a = {&flags_[s], token(sl.req, sl.phase)};
        const acs_seg wr[1] = {{(uint64_t)(uintptr_t)&flags_[s], 8}};
        return submit(sl, ACS_K_SIGNAL, r, nr, wr, 1, &a, sizeof(a));
    }

    int admit(int32_t i, uint64_t block, uint64_t bytes, double t_admit)
    {
        const int32_t s = free_slots_.back();
        free_slots_.pop_back();
        Slot &sl = slots_[(size_t)s];
        sl.req = i;
        sl.group = pick_group();
        sl.block = block;
        sl.bytes = bytes;
        load_[(size_t)sl.group]++;
        resident_.push_back(s);
        uint64_t used = 0;
        (void)acs_pool_info(pool_, &used, nullptr, nullptr);
        if (used > stats_.peak_pool_bytes) stats_.peak_pool_bytes = used;
        if (resident_.size() > stats_.peak_resident) stats_.peak_resident = resident_.size();
        const acs_serve_request &q = req_[i];
        if (res_) {
            res_[i].admit_ns = t_admit;
            res_[i].done_ns = -1;
            res_[i].kernels = 0;
            res_[i].footprint = bytes;
            res_[i].group = sl.group;
            res_[i].multi_islands = -1;
        }
        if (q.kind == ACS_SERVE_RL) return admit_rl(s, sl, q);
        return admit_dnn(s, sl, q);
    }

    int admit_rl(int32_t s, Slot &sl, const acs_serve_request &q)
    {
        uint64_t off[ACS_RL_NREGIONS];
        acs::rl_offsets(q.n, off);
        sl.scene = {};
        sl.scene.n = q.n;
        sl.scene.iters = q.iters;
        sl.scene.r = q.r;
        sl.scene.dt = q.dt;
        sl.scene.arena = sl.block;
        sl.scene.plan = reinterpret_cast<int32_t *>(plans_ + kPlanSlotBytes * (size_t)s);
        sl.counts = {};
        sl.rl = std::make_unique<acs::RLStep>(w_, sl.group, &sl.scene);
        sl.phase = 1;
        // stage the input image (X and V at their arena offsets)
        const uint64_t img = off[ACS_RL_V] + 16ull * (uint64_t)q.n;
        {
            const acs_args_copy a = {reinterpret_cast<void *>(sl.block), reinterpret_cast<const void *>(q.input), img};
            const acs_seg r[1] = {{q.input, img}};
            const acs_seg wr[1] = {{sl.block, img}};
            if (int rc = submit(sl, ACS_K_COPY, r, 1, wr, 1, &a, sizeof(a))) return rc;
        }
        const uint64_t before = sl.counts.kernels;
        if (int rc = sl.rl->submit_prefix(sl.counts)) return rc;
        count(sl, sl.counts.kernels - before);
        const acs_seg r[1] = {{(uint64_t)(uintptr_t)sl.scene.plan, 4 * acs::rl_plan_ints(q.n)}};
        return signal(sl, s, r, 1);
    }

    int submit_rl_tail(int32_t s)
    {
        Slot &sl = slots_[(size_t)s];
        const acs_serve_request &q = req_[sl.req];
        const uint64_t before = sl.counts.kernels;
        if (int rc = sl.rl->submit_tail(sl.counts)) return rc;
        count(sl, sl.counts.kernels - before);
        if (res_) res_[sl.req].multi_islands = (int32_t)sl.counts.multi_islands;
        uint64_t off[ACS_RL_NREGIONS];
        acs::rl_offsets(q.n, off);
        const uint64_t img = off[ACS_RL_V] + 16ull * (uint64_t)q.n;
        {
            const acs_args_copy a = {reinterpret_cast<void *>(q.output), reinterpret_cast<const void *>(sl.block), img};
            const acs_seg r[1] = {{sl.block, img}};
            const acs_seg wr[1] = {{q.output, img}};
            if (int rc = submit(sl, ACS_K_COPY, r, 1, wr, 1, &a, sizeof(a))) return rc;
        }
        sl.phase = 2;
        const acs_seg r[2] = {{sl.block, sl.bytes}, {q.output, img}};
        return signal(sl, s, r, 2);
    }

    int admit_dnn(int32_t s, Slot &sl, const acs_serve_request &q)
    {
        acs_dnn_graph g = *cfg_.model;
        g.x = reinterpret_cast<const float *>(q.input);
        uint64_t p = sl.block;
        for (int32_t c = 0; c < g.n_cells; c++) {
            acs_dnn_cell &L = g.cell[c];
            const uint64_t hout = (uint64_t)(L.hin / (L.stride > 0 ? L.stride : 1));
            const uint64_t t = acs::rl_align(4 * hout * hout * (uint64_t)L.cout);
            L.t3 = reinterpret_cast<float *>(p);
            L.t1 = reinterpret_cast<float *>(p + t);
            L.y = reinterpret_cast<float *>(p + 2 * t);
            p += 3 * t;
        }
        g.pool = reinterpret_cast<float *>(p);
        g.out = reinterpret_cast<float *>(q.output);
        sl.phase = 2;
        uint64_t k = 0;
        if (int rc = acs::dnn_submit_group(w_, sl.group, &g, q.logits, &k)) return rc;
        count(sl, k);
        const acs_seg r[2] = {{sl.block, sl.bytes}, {q.output, 4ull * (uint64_t)g.classes}};
        return signal(sl, s, r, 2);
    }

    acs_window *w_;
    acs_serve_config cfg_;
    const acs_serve_request *req_;
    int32_t n_;
    acs_serve_result *res_;
    int32_t groups_ = 1;
    acs_pool *pool_ = nullptr;
    uint64_t *flags_ = nullptr;
    uint8_t *plans_ = nullptr;
    std::vector<Slot> slots_;
    std::vector<int32_t> free_slots_, resident_, load_;
    acs_serve_stats stats_ = {};
};

}  // namespace

extern "C" uint64_t acs_serve_host_bytes(int32_t max_resident)
{
    return max_resident < 1 ? 0 : host_bytes(max_resident);
}

extern "C" int acs_serve_run(acs_window *w, const acs_serve_config *cfg, const acs_serve_request *req, int32_t n_req,
                             acs_serve_result *res, acs_serve_stats *stats)
{
    if (!w || !cfg || n_req < 0 || (n_req > 0 && !req)) return ACS_EINVAL;
    Server sv(w, *cfg, req, n_req, res);
    if (int rc = sv.validate()) return rc;
    if (int rc = sv.setup()) return rc;
    return sv.run(stats);
}
