// Native application drivers for the synthetic workloads (acs_workloads.h).
// They use the public API only; the range helpers below are the workload's
// get_addresses functions (Section IV-A): they state, from the launch
// arguments, which bytes each kernel reads and writes.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <vector>

#include "acs.h"
#include "acs_tasks.h"
#include "acs_workloads.h"
#include "rl_layout.hpp"

namespace {

double wall_ns()
{
    return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

extern "C" {

void *acs_host_alloc(size_t bytes)
{
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) return nullptr;
    return p;
}

int acs_host_free(void *p)
{
    if (!p) return ACS_OK;
    return hipHostFree(p) == hipSuccess ? ACS_OK : ACS_EDEVICE;
}

}  // extern "C"

namespace {

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
        const acs_seg plan_seg = {(uint64_t)(uintptr_t)sc_->plan, 4ull * acs::rl_plan_ints(sc_->n)};
        a_.iter = a_.b0 = a_.b1 = 0;
        {
            const acs_seg r[2] = {region(ACS_RL_X), region(ACS_RL_V)};
            const acs_seg wr[1] = {region(ACS_RL_P)};
            if (int rc = submit(ACS_K_RL_PREDICT, r, 2, wr, 1, cnt)) return rc;
        }
        {
            const acs_seg r[1] = {region(ACS_RL_P)};
            const acs_seg wr[1] = {span(ACS_RL_DEG, ACS_RL_LABEL)};
            if (int rc = submit(ACS_K_RL_BROADPHASE, r, 1, wr, 1, cnt)) return rc;
        }
        {
            const acs_seg r[1] = {span(ACS_RL_DEG, ACS_RL_LABEL)};
            const acs_seg wr[2] = {span(ACS_RL_LABEL, ACS_RL_END), plan_seg};
            if (int rc = submit(ACS_K_RL_ISLANDS, r, 1, wr, 2, cnt)) return rc;
        }
        const acs_seg r[2] = {region(ACS_RL_P), region(ACS_RL_PERM)};
        const acs_seg wr[1] = {region(ACS_RL_Q0)};
        return submit(ACS_K_RL_PERMUTE, r, 2, wr, 1, cnt);
    }

    // after the prefix has completed: the plan's Jacobi kernels
    // (iteration-major) and integrate
    int submit_tail(acs_rl_counts &cnt)
    {
        const int32_t *plan = (const int32_t *)sc_->plan;
        const int32_t nmulti = __atomic_load_n(&plan[1], __ATOMIC_ACQUIRE);
        if (nmulti < 0 || nmulti > sc_->n / 2) return ACS_EKERNEL;
        cnt.steps++;
        cnt.islands += (uint64_t)plan[0];
        cnt.multi_islands += (uint64_t)nmulti;
        cnt.edges += (uint64_t)plan[2];
        for (int32_t it = 0; it < sc_->iters; it++) {
            const int src = (it % 2 == 0) ? ACS_RL_Q0 : ACS_RL_Q1, dst = (it % 2 == 0) ? ACS_RL_Q1 : ACS_RL_Q0;
            for (int32_t k = 0; k < nmulti; k++) {
                const int32_t b0 = plan[4 + 4 * k], b1 = plan[5 + 4 * k], e0 = plan[6 + 4 * k], e1 = plan[7 + 4 * k];
                if (b0 < 0 || b1 > sc_->n || b1 - b0 < 2 || e0 < 0 || e1 < e0 || e1 > sc_->n * (sc_->n - 1))
                    return ACS_EKERNEL;   // a plan row the islands kernel cannot produce
                a_.iter = it;
                a_.b0 = b0;
                a_.b1 = b1;
                const acs_seg r[3] = {vec(src, b0, b1), ints(ACS_RL_PADJ_OFF, b0, b1 + 1), ints(ACS_RL_PADJ, e0, e1)};
                const acs_seg wr[1] = {vec(dst, b0, b1)};
                if (int rc = submit(ACS_K_RL_JACOBI, r, 3, wr, 1, cnt)) return rc;
                cnt.jacobi_kernels++;
                cnt.jacobi_bodies += (uint64_t)(b1 - b0);
                cnt.jacobi_edges += (uint64_t)(e1 - e0);
            }
        }
        a_.iter = a_.b0 = a_.b1 = 0;
        const acs_seg r[4] = {region(ACS_RL_P), region(ACS_RL_V), region(ACS_RL_Q0), region(ACS_RL_INV_PERM)};
        const acs_seg wr[2] = {region(ACS_RL_X), region(ACS_RL_V)};
        return submit(ACS_K_RL_INTEGRATE, r, 4, wr, 2, cnt);
    }

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
};

bool scene_ok(const acs_rl_scene *sc)
{
    return sc && sc->n >= 2 && sc->n <= acs::kRLMaxBodies && sc->plan && sc->iters >= 0;
}

}  // namespace

extern "C" {

int acs_rl_run(acs_window *w, const acs_rl_scene *sc, int32_t steps, double *step_ns, acs_rl_counts *counts)
{
    if (!w || !scene_ok(sc) || steps < 0) return ACS_EINVAL;
    RLStep s(w, 0, sc);
    acs_rl_counts cnt = {};
    double t_prev = wall_ns();
    for (int32_t step = 0; step < steps; step++) {
        if (int rc = s.submit_prefix(cnt)) return rc;
        // the island list is known only now: drain, read the plan
        if (int rc = acs_sync(w)) return rc;
        const double t_now = wall_ns();
        if (step_ns && step > 0) step_ns[step - 1] = t_now - t_prev;
        t_prev = t_now;
        if (int rc = s.submit_tail(cnt)) return rc;
    }
    const int rc = acs_sync(w);
    const double t_end = wall_ns();
    if (step_ns && steps > 0) step_ns[steps - 1] = t_end - t_prev;
    if (counts) *counts = cnt;
    return rc;
}

int acs_rl_run_batch(acs_window *w, const acs_rl_scene *scenes, int32_t n_scenes, int32_t n_groups, int32_t steps,
                     double *step_ns, acs_rl_counts *counts)
{
    if (!w || !scenes || n_scenes < 1 || n_groups < 1 || n_groups > 8 || steps < 0) return ACS_EINVAL;
    std::vector<RLStep> st;
    st.reserve((size_t)n_scenes);
    for (int32_t i = 0; i < n_scenes; i++) {
        if (!scene_ok(&scenes[i])) return ACS_EINVAL;
        st.emplace_back(w, i % n_groups, &scenes[i]);
    }
    acs_rl_counts cnt = {};
    for (int32_t step = 0; step < steps; step++) {
        const double t0 = wall_ns();
        for (auto &s : st)
            if (int rc = s.submit_prefix(cnt)) return rc;
        // group by group: once a group has drained, its scenes' plans are
        // readable; the other groups keep running meanwhile
        for (int32_t g = 0; g < n_groups; g++) {
            if (int rc = acs_sync_group(w, g, 0)) return rc;
            for (int32_t i = g; i < n_scenes; i += n_groups)
                if (int rc = st[(size_t)i].submit_tail(cnt)) return rc;
        }
        if (step == steps - 1 || step_ns) {
            if (int rc = acs_sync(w)) return rc;
        }
        if (step_ns) step_ns[step] = wall_ns() - t0;
    }
    if (counts) *counts = cnt;
    return ACS_OK;
}

int acs_nop_run(acs_window *w, int32_t n, int32_t chain, uint64_t spin_ns, double *out_ns)
{
    if (!w || n < 0) return ACS_EINVAL;
    static uint8_t dummy[1 << 16];
    const uint64_t base = (uint64_t)(uintptr_t)dummy;
    acs_args_nop a = {spin_ns};
    const double t0 = wall_ns();
    for (int32_t i = 0; i < n; i++) {
        const acs_seg s = {chain ? base : base + (uint64_t)(i % (1 << 16)), 1};
        const int rc = acs_submit(w, ACS_K_NOP, chain ? &s : nullptr, chain ? 1 : 0, &s, 1, &a, sizeof(a), nullptr);
        if (rc != ACS_OK) return rc;
    }
    const int rc = acs_sync(w);
    if (out_ns) *out_ns = wall_ns() - t0;
    return rc;
}

int acs_dnn_submit(acs_window *w, const acs_dnn_graph *g, const float *logits, uint64_t *n_kernels)
{
    if (!w || !g || !logits || g->n_cells < 1 || g->n_cells > ACS_DNN_MAX_CELLS || g->classes < 1 || !g->x ||
        !g->pool || !g->fc_w || !g->fc_b || !g->out)
        return ACS_EINVAL;
    auto seg = [](const void *p, uint64_t bytes) { return acs_seg{(uint64_t)(uintptr_t)p, bytes}; };
    uint64_t kernels = 0;
    const float *cur = g->x;
    uint64_t cur_bytes = 4ull * g->cell[0].hin * g->cell[0].hin * g->cell[0].cin;
    int32_t cur_c = g->cell[0].cin, cur_h = g->cell[0].hin;
    for (int32_t c = 0; c < g->n_cells; c++) {
        const acs_dnn_cell &L = g->cell[c];
        if (L.hin != cur_h || L.cin != cur_c || (L.stride != 1 && L.stride != 2) || L.hin % L.stride != 0)
            return ACS_EINVAL;
        const int32_t hout = L.hin / L.stride;
        const uint64_t out_bytes = 4ull * hout * hout * L.cout;
        const bool g3 = logits[2 * c] > 0.0f, g1 = logits[2 * c + 1] > 0.0f || L.stride == 2;
        const float *parts[2];
        int np = 0;
        if (g3) {
            acs_args_conv a = {cur, L.w3, L.b3, L.t3, L.hin, L.cin, L.cout, 3, L.stride};
            const acs_seg r[3] = {seg(cur, cur_bytes), seg(L.w3, 36ull * L.cin * L.cout), seg(L.b3, 4ull * L.cout)};
            const acs_seg wr[1] = {seg(L.t3, out_bytes)};
            if (int rc = acs_submit(w, ACS_K_CONV, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
            parts[np++] = L.t3;
            kernels++;
        }
        if (g1) {
            acs_args_conv a = {cur, L.w1, L.b1, L.t1, L.hin, L.cin, L.cout, 1, L.stride};
            const acs_seg r[3] = {seg(cur, cur_bytes), seg(L.w1, 4ull * L.cin * L.cout), seg(L.b1, 4ull * L.cout)};
            const acs_seg wr[1] = {seg(L.t1, out_bytes)};
            if (int rc = acs_submit(w, ACS_K_CONV, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
            parts[np++] = L.t1;
            kernels++;
        }
        if (np > 0) {
            acs_args_join a = {L.y, parts[0], np > 1 ? parts[1] : nullptr, (uint32_t)(out_bytes / 4)};
            const acs_seg r[2] = {seg(parts[0], out_bytes), seg(np > 1 ? parts[1] : nullptr, np > 1 ? out_bytes : 0)};
            const acs_seg wr[1] = {seg(L.y, out_bytes)};
            if (int rc = acs_submit(w, ACS_K_JOIN, r, np, wr, 1, &a, sizeof(a), nullptr)) return rc;
            kernels++;
            cur = L.y;
            cur_bytes = out_bytes;
            cur_h = hout;
            cur_c = L.cout;
        } else if (L.stride != 1 || L.cout != L.cin) {
            return ACS_EINVAL;   // unreachable: a cell that changes shape always runs its 1x1 branch
        }
    }
    {
        acs_args_avgpool a = {g->pool, cur, cur_h * cur_h, cur_c};
        const acs_seg r[1] = {seg(cur, cur_bytes)};
        const acs_seg wr[1] = {seg(g->pool, 4ull * cur_c)};
        if (int rc = acs_submit(w, ACS_K_AVGPOOL, r, 1, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    {
        acs_args_fc a = {g->out, g->pool, g->fc_w, g->fc_b, cur_c, g->classes};
        const acs_seg r[3] = {seg(g->pool, 4ull * cur_c), seg(g->fc_w, 4ull * cur_c * g->classes),
                              seg(g->fc_b, 4ull * g->classes)};
        const acs_seg wr[1] = {seg(g->out, 4ull * g->classes)};
        if (int rc = acs_submit(w, ACS_K_FC, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    if (n_kernels) *n_kernels = kernels;
    return ACS_OK;
}

}  // extern "C"
