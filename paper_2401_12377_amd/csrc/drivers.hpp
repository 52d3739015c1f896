// Application-side graph builders shared by the native drivers (the RL
// step and the gated network); they call the public API only.  The range
// helpers are the workload's get_addresses functions (Section IV-A): they
// state, from the launch arguments, which bytes each kernel reads and writes.
#pragma once
#include <stdint.h>

#include <chrono>
#include <immintrin.h>

#include "acs.h"
#include "acs_tasks.h"
#include "acs_workloads.h"
#include "rl_layout.hpp"

namespace acs {

// One scene's kernels of a step, in the two halves the host submits
// (before and after reading the input-dependent island plan).
class RLStep {
public:
    RLStep(acs_window *w, int32_t group, const acs_rl_scene *sc) : w_(w), g_(group), sc_(sc)
    {
        acs::rl_offsets(sc->n, off_);
        a_ = {};
        a_.base = sc->arena;
        a_.plan = (uint64_t)(uintptr_t)sc->plan;
        a_.n = sc->n;
        a_.r = sc->r;
        a_.dt = sc->dt;
    }

    // predict, broadphase, islands, permute
    int submit_prefix(acs_rl_counts &cnt)
    {
        for (int k = 0; k < 4; k++)
            if (int rc = submit_stage(k, cnt)) return rc;
        return ACS_OK;
    }

    // kernel k of the first half: 0 predict, 1 broadphase, 2 islands, 3 permute
    int submit_stage(int k, acs_rl_counts &cnt)
    {
        a_.iter = a_.b0 = a_.b1 = 0;
        if (k == 0) {
            const acs_seg r[2] = {region(ACS_RL_X), region(ACS_RL_V)};
            const acs_seg wr[1] = {region(ACS_RL_P)};
            return submit(ACS_K_RL_PREDICT, r, 2, wr, 1, cnt);
        }
        if (k == 1) {
            const acs_seg r[1] = {region(ACS_RL_P)};
            const acs_seg wr[1] = {span(ACS_RL_DEG, ACS_RL_LABEL)};
            return submit(ACS_K_RL_BROADPHASE, r, 1, wr, 1, cnt);
        }
        if (k == 2) {
            const acs_seg plan_seg = {(uint64_t)(uintptr_t)sc_->plan, 4ull * acs::rl_plan_ints(sc_->n)};
            const acs_seg r[1] = {span(ACS_RL_DEG, ACS_RL_LABEL)};
            const acs_seg wr[2] = {span(ACS_RL_LABEL, ACS_RL_END), plan_seg};
            // The islands kernel stores this stamp into plan[3] after the
            // rest of the plan.  No kernel is writing the plan now (the last
            // islands kernel of this scene has been waited for), so the old
            // stamp is cleared first and never mistaken for the new one.
            stamp_ = stamp_ >= 0x7FFFFFFF ? 1 : stamp_ + 1;
            __atomic_store_n(&((int32_t *)sc_->plan)[3], 0, __ATOMIC_RELAXED);
            a_.iter = stamp_;
            const int rc = submit(ACS_K_RL_ISLANDS, r, 1, wr, 2, cnt);
            a_.iter = 0;
            return rc;
        }
        const acs_seg r[2] = {region(ACS_RL_P), region(ACS_RL_PERM)};
        const acs_seg wr[1] = {region(ACS_RL_Q0)};
        return submit(ACS_K_RL_PERMUTE, r, 2, wr, 1, cnt);
    }

    // once the plan is readable: the plan's Jacobi kernels
    // (iteration-major) and integrate
    int submit_tail(acs_rl_counts &cnt)
    {
        if (int rc = tail_begin(cnt)) return rc;
        for (int32_t it = 0; it < sc_->iters; it++)
            if (int rc = submit_iteration(it, cnt)) return rc;
        return submit_integrate(cnt);
    }

    // True once the islands kernel of this step has published the plan (no
    // wait).  On the device-resident path the plan reaches host memory after
    // the islands kernel has completed, so a completion alone does not say
    // that the plan is readable; its stamp does.
    bool plan_ready() const
    {
        return __atomic_load_n(&((const int32_t *)sc_->plan)[3], __ATOMIC_ACQUIRE) == stamp_;
    }

    // Waits until the islands kernel of this step has published the plan
    // (its stamp in plan[3]) while the window keeps running: the host needs
    // the island list before it can state the rest of the step, but not an
    // empty window.  acs_poll keeps a host-side window dispatching and
    // reports a failed window; a minute without the stamp is a time-out.
    int wait_plan()
    {
        const int32_t *stamp = &((const int32_t *)sc_->plan)[3];
        auto t0 = std::chrono::steady_clock::now();
        for (uint32_t spin = 0;; spin++) {
            if (__atomic_load_n(stamp, __ATOMIC_ACQUIRE) == stamp_) return ACS_OK;
            if ((spin & 15u) == 0)
                if (int rc = acs_poll(w_)) return rc;
            if ((spin & 0xFFFFu) == 0xFFFFu && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60))
                return ACS_ETIMEDOUT;
            _mm_pause();
        }
    }

    // Reads and checks the island plan (once the islands kernel published it).
    int tail_begin(acs_rl_counts &cnt)
    {
        const int32_t *plan = (const int32_t *)sc_->plan;
        const int32_t nmulti = __atomic_load_n(&plan[1], __ATOMIC_ACQUIRE);
        if (nmulti < 0 || nmulti > sc_->n / 2) return ACS_EKERNEL;
        for (int32_t k = 0; k < nmulti; k++) {
            const int32_t b0 = plan[4 + 4 * k], b1 = plan[5 + 4 * k], e0 = plan[6 + 4 * k], e1 = plan[7 + 4 * k];
            if (b0 < 0 || b1 > sc_->n || b1 - b0 < 2 || e0 < 0 || e1 < e0 || e1 > sc_->n * (sc_->n - 1))
                return ACS_EKERNEL;   // a plan row the islands kernel cannot produce
        }
        nmulti_ = nmulti;
        cnt.steps++;
        cnt.islands += (uint64_t)plan[0];
        cnt.multi_islands += (uint64_t)nmulti;
        cnt.edges += (uint64_t)plan[2];
        return ACS_OK;
    }

    // Jacobi iteration `it` over every multi-body island (after tail_begin)
    int submit_iteration(int32_t it, acs_rl_counts &cnt)
    {
        for (int32_t k = 0; k < nmulti_; k++)
            if (int rc = submit_island(it, k, cnt)) return rc;
        return ACS_OK;
    }

    // Jacobi iteration `it` over multi-body island k of the plan (after
    // tail_begin; k < multi())
    int submit_island(int32_t it, int32_t k, acs_rl_counts &cnt)
    {
        const int32_t *plan = (const int32_t *)sc_->plan;
        const int src = (it % 2 == 0) ? ACS_RL_Q0 : ACS_RL_Q1, dst = (it % 2 == 0) ? ACS_RL_Q1 : ACS_RL_Q0;
        const int32_t b0 = plan[4 + 4 * k], b1 = plan[5 + 4 * k], e0 = plan[6 + 4 * k], e1 = plan[7 + 4 * k];
        a_.iter = it;
        a_.b0 = b0;
        a_.b1 = b1;
        const acs_seg r[3] = {vec(src, b0, b1), ints(ACS_RL_PADJ_OFF, b0, b1 + 1), ints(ACS_RL_PADJ, e0, e1)};
        const acs_seg wr[1] = {vec(dst, b0, b1)};
        if (int rc = submit(ACS_K_RL_JACOBI, r, 3, wr, 1, cnt)) return rc;
        cnt.jacobi_kernels++;
        cnt.jacobi_bodies += (uint64_t)(b1 - b0);
        cnt.jacobi_edges += (uint64_t)(e1 - e0);
        return ACS_OK;
    }

    // multi-body islands of the plan read by tail_begin
    int32_t multi() const { return nmulti_; }

    int submit_integrate(acs_rl_counts &cnt)
    {
        a_.iter = a_.b0 = a_.b1 = 0;
        const acs_seg r[4] = {region(ACS_RL_P), region(ACS_RL_V), region(ACS_RL_Q0), region(ACS_RL_INV_PERM)};
        const acs_seg wr[2] = {region(ACS_RL_X), region(ACS_RL_V)};
        return submit(ACS_K_RL_INTEGRATE, r, 4, wr, 2, cnt);
    }

    int32_t iters() const { return sc_->iters; }

private:
    acs_seg region(int r) const { return acs_seg{sc_->arena + off_[r], off_[r + 1] - off_[r]}; }
    acs_seg span(int r0, int r1) const { return acs_seg{sc_->arena + off_[r0], off_[r1] - off_[r0]}; }
    acs_seg vec(int r, int32_t b0, int32_t b1) const
    {
        return acs_seg{sc_->arena + off_[r] + 16ull * b0, 16ull * (uint64_t)(b1 - b0)};
    }
    acs_seg ints(int r, int32_t b0, int32_t b1) const
    {
        return acs_seg{sc_->arena + off_[r] + 4ull * b0, 4ull * (uint64_t)(b1 - b0)};
    }
    int submit(int32_t kid, const acs_seg *r, int32_t nr, const acs_seg *wr, int32_t nw, acs_rl_counts &cnt)
    {
        const int rc = acs_submit_group(w_, g_, kid, r, nr, wr, nw, &a_, sizeof(a_), nullptr);
        if (rc == ACS_OK) cnt.kernels++;
        return rc;
    }

    acs_window *w_;
    int32_t g_;
    const acs_rl_scene *sc_;
    uint64_t off_[ACS_RL_NREGIONS];
    acs_args_rl a_;
    int32_t nmulti_ = 0;
    int32_t stamp_ = 0;   // of the last islands kernel submitted
};

// Submits one inference of the gated network into window group `group`
// (acs_dnn_submit is this with group 0).
int dnn_submit_group(acs_window *w, int32_t group, const acs_dnn_graph *g, const float *logits, uint64_t *n_kernels);

// Device bytes of the activations of one inference (every cell's two branch
// outputs and output, and the pooled vector), each 256-byte aligned.
uint64_t dnn_activation_bytes(const acs_dnn_graph *g);

}  // namespace acs
