// Native application drivers for the synthetic workloads (acs_workloads.h).
// They use the public API only; the range helpers below are the workload's
// get_addresses functions (Section IV-A): they state, from the launch
// arguments, which bytes each kernel reads and writes.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "acs.h"
#include "acs_tasks.h"
#include "acs_workloads.h"
#include "drivers.hpp"
#include "rl_layout.hpp"

namespace {

double wall_ns()
{
    return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

namespace {

// Jacobi sweeps alternate Q0 -> Q1 -> Q0 and integrate reads Q0: an odd
// sweep count would leave the last sweep's result unread, so it is refused.
bool scene_ok(const acs_rl_scene *sc)
{
    return sc && sc->n >= 2 && sc->n <= acs::kRLMaxBodies && sc->plan && sc->iters >= 0 && sc->iters % 2 == 0;
}

// The ranges of probe kernel k (k < 2048), 64 bytes each, the first half
// reads and the rest writes: the first range in a low strip and the last in
// a high strip (64-byte slots indexed by k), the others 4 KiB apart in a
// block of 1 MiB of the kernel's own between the strips.  No two kernels
// share a byte, every kernel's bounding interval meets every other's (so
// every pair of ranges is tested), and merging ranges beyond the eight a
// kernel keeps joins the nearest ones, inside the kernel's own block.
void probe_segs(uint64_t base, int32_t k, int32_t nsegs, std::vector<acs_seg> &r, std::vector<acs_seg> &wr)
{
    r.clear();
    wr.clear();
    for (int32_t s = 0; s < nsegs; s++) {
        uint64_t at;
        if (s == 0)
            at = base + 64ull * (uint64_t)k;
        else if (s == nsegs - 1)
            at = base + (4ull << 30) + 64ull * (uint64_t)k;
        else
            at = base + (1ull << 20) * (1ull + (uint64_t)k) + 4096ull * (uint64_t)s;
        (s < nsegs / 2 ? r : wr).push_back(acs_seg{at, 64});
    }
}

}  // namespace

extern "C" {

int acs_rl_run(acs_window *w, const acs_rl_scene *sc, int32_t steps, double *step_ns, acs_rl_counts *counts)
{
    if (!w || !scene_ok(sc) || steps < 0) return ACS_EINVAL;
    acs::RLStep s(w, 0, sc);
    acs_rl_counts cnt = {};
    double t_prev = wall_ns();
    for (int32_t step = 0; step < steps; step++) {
        if (int rc = s.submit_prefix(cnt)) return rc;
        // the island list is known only once the islands kernel has run
        if (int rc = s.wait_plan()) return rc;
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
    std::vector<acs::RLStep> st;
    st.reserve((size_t)n_scenes);
    for (int32_t i = 0; i < n_scenes; i++) {
        if (!scene_ok(&scenes[i])) return ACS_EINVAL;
        st.emplace_back(w, i % n_groups, &scenes[i]);
    }
    int32_t max_iters = 0;
    for (auto &s : st) max_iters = std::max(max_iters, s.iters());
    acs_rl_counts cnt = {};
    for (int32_t step = 0; step < steps; step++) {
        const double t0 = wall_ns();
        // Scenes are independent, so their kernels may come in any
        // interleaving; stage by stage across the scenes puts kernels of
        // different scenes next to each other in the window, all ready.
        for (int k = 0; k < 4; k++)
            for (auto &s : st)
                if (int rc = s.submit_stage(k, cnt)) return rc;
        // group by group: once its scenes' plans are published, Jacobi
        // iteration by iteration across the group's scenes, then integrate;
        // the window keeps running meanwhile.
        for (int32_t g = 0; g < n_groups; g++) {
            for (int32_t i = g; i < n_scenes; i += n_groups)
                if (int rc = st[(size_t)i].wait_plan()) return rc;
            for (int32_t i = g; i < n_scenes; i += n_groups)
                if (int rc = st[(size_t)i].tail_begin(cnt)) return rc;
            // island by island across the scenes, so that the kernels next
            // to each other touch different scenes' memory: the dependency
            // check then drops them on their bounding intervals alone
            int32_t max_multi = 0;
            for (int32_t i = g; i < n_scenes; i += n_groups) max_multi = std::max(max_multi, st[(size_t)i].multi());
            for (int32_t it = 0; it < max_iters; it++)
                for (int32_t k = 0; k < max_multi; k++)
                    for (int32_t i = g; i < n_scenes; i += n_groups)
                        if (it < st[(size_t)i].iters() && k < st[(size_t)i].multi())
                            if (int rc = st[(size_t)i].submit_island(it, k, cnt)) return rc;
            for (int32_t i = g; i < n_scenes; i += n_groups)
                if (int rc = st[(size_t)i].submit_integrate(cnt)) return rc;
        }
        if (step == steps - 1 || step_ns) {
            if (int rc = acs_sync(w)) return rc;
        }
        if (step_ns) step_ns[step] = wall_ns() - t0;
    }
    if (counts) *counts = cnt;
    return ACS_OK;
}

int acs_rl_run_graphs(const acs_rl_scene *sc, int32_t steps, int32_t device, double *step_ns, acs_rl_counts *counts,
                      double *build_ns)
{
    if (!scene_ok(sc) || steps < 0) return ACS_EINVAL;
    // a window that only records: its own stream never runs anything
    acs_window *w = acs_window_create(ACS_W_MAX);
    if (!w) return acs_last_error();
    acs_config cfg;
    acs_config_default(&cfg);
    cfg.path = ACS_PATH_INORDER;
    cfg.device = device;
    int rc = acs_window_configure(w, &cfg);
    acs::RLStep s(w, 0, sc);
    acs_rl_counts cnt = {};
    double built = 0;
    // one half of a step: record, build, run, wait, destroy
    auto half = [&](bool tail) -> int {
        const double t0 = wall_ns();
        if (int r = acs_graph_begin(w)) return r;
        int r = tail ? s.submit_tail(cnt) : s.submit_prefix(cnt);
        acs_graph *g = nullptr;
        const int re = acs_graph_end(w, &g);
        if (r == ACS_OK) r = re;
        built += wall_ns() - t0;
        if (r != ACS_OK) {
            acs_graph_destroy(g);
            return r;
        }
        r = acs_graph_launch(g);
        if (r == ACS_OK) r = acs_graph_sync(g);
        acs_graph_destroy(g);
        return r;
    };
    for (int32_t step = 0; rc == ACS_OK && step < steps; step++) {
        const double t0 = wall_ns();
        rc = half(false);
        if (rc == ACS_OK) rc = half(true);
        if (step_ns) step_ns[step] = wall_ns() - t0;
    }
    acs_window_destroy(w);
    if (counts) *counts = cnt;
    if (build_ns) *build_ns = built;
    return rc;
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

int acs_nop_segs_run(acs_window *w, int32_t n, int32_t nsegs, double *out_ns)
{
    if (!w || n < 0 || nsegs < 1 || nsegs > 64) return ACS_EINVAL;
    acs_args_nop a = {0};
    std::vector<acs_seg> r, wr;
    const double t0 = wall_ns();
    for (int32_t i = 0; i < n; i++) {
        // in an address range nothing touches (no body reads them)
        probe_segs(1ull << 40, i % 2048, nsegs, r, wr);
        const int rc = acs_submit(w, ACS_K_NOP, r.data(), (int32_t)r.size(), wr.data(), (int32_t)wr.size(), &a, sizeof(a), nullptr);
        if (rc != ACS_OK) return rc;
    }
    const int rc = acs_sync(w);
    if (out_ns) *out_ns = wall_ns() - t0;
    return rc;
}

int acs_check_probe(int32_t W, int32_t nsegs, int32_t reps, double *ns_checked, double *ns_empty, double *tests_out)
{
    if (W < 2 || W > ACS_W_MAX || nsegs < 2 || nsegs > 64 || reps < 1 || !ns_checked || !ns_empty) return ACS_EINVAL;
    auto segs = [&](int32_t k, std::vector<acs_seg> &r, std::vector<acs_seg> &wr) { probe_segs(1ull << 32, k, nsegs, r, wr); };
    acs_args_nop a = {0};
    double result[2] = {0, 0};
    double tests = 0;
    for (int pass = 0; pass < 2; pass++) {
        acs_window *w = acs_window_create(W);
        if (!w) return acs_last_error();
        acs_config cfg;
        acs_config_default(&cfg);
        cfg.path = ACS_PATH_MANUAL;
        cfg.queue_depth = 4096;
        int rc = acs_window_configure(w, &cfg);
        std::vector<acs_seg> r, wr;
        const int32_t resident = pass == 0 ? W - 1 : 0;
        for (int32_t k = 0; rc == ACS_OK && k < resident; k++) {
            segs(k, r, wr);
            rc = acs_submit(w, ACS_K_NOP, r.data(), (int32_t)r.size(), wr.data(), (int32_t)wr.size(), &a, sizeof(a), nullptr);
        }
        // the resident kernels are taken (executing) and never completed
        uint64_t taken[ACS_W_MAX];
        int32_t nt = 0;
        if (rc == ACS_OK && resident > 0) rc = acs_manual_take_ready(w, taken, ACS_W_MAX, &nt);
        acs_stats s0 = {}, s1 = {};
        if (rc == ACS_OK) rc = acs_stats_get(w, &s0);
        const double t0 = wall_ns();
        for (int32_t i = 0; rc == ACS_OK && i < reps; i++) {
            segs(W + i % 1024, r, wr);
            uint64_t seq = 0, got = 0;
            int32_t n = 0;
            rc = acs_submit(w, ACS_K_NOP, r.data(), (int32_t)r.size(), wr.data(), (int32_t)wr.size(), &a, sizeof(a), &seq);
            if (rc == ACS_OK) rc = acs_manual_take_ready(w, &got, 1, &n);
            if (rc == ACS_OK && (n != 1 || got != seq)) rc = ACS_EKERNEL;
            if (rc == ACS_OK) rc = acs_manual_complete(w, seq, 0);
        }
        const double t1 = wall_ns();
        if (rc == ACS_OK) rc = acs_stats_get(w, &s1);
        if (rc == ACS_OK && pass == 0) tests = (double)(s1.overlap_tests - s0.overlap_tests) / reps;
        for (int32_t q = 0; q < nt; q++) (void)acs_manual_complete(w, taken[q], 0);
        acs_window_destroy(w);
        if (rc != ACS_OK) return rc;
        result[pass] = (t1 - t0) / reps;
    }
    *ns_checked = result[0];
    *ns_empty = result[1];
    if (tests_out) *tests_out = tests;
    return ACS_OK;
}

int acs_dnn_submit(acs_window *w, const acs_dnn_graph *g, const float *logits, uint64_t *n_kernels)
{
    return acs::dnn_submit_group(w, 0, g, logits, n_kernels);
}

int acs_dag_submit(acs_window *w, const acs_dag_graph *g, uint64_t *n_kernels)
{
    if (!w || !g || g->n_nodes < 1 || g->n_nodes > ACS_DAG_MAX_NODES || g->h < 1 || g->c < 1 || g->classes < 1 || !g->x ||
        !g->sink || !g->pool || !g->fc_w || !g->fc_b || !g->out)
        return ACS_EINVAL;
    const uint64_t act = 4ull * (uint64_t)g->h * (uint64_t)g->h * (uint64_t)g->c;
    const uint32_t n_act = (uint32_t)(act / 4);
    auto seg = [](const void *p, uint64_t bytes) { return acs_seg{(uint64_t)(uintptr_t)p, bytes}; };
    uint64_t kernels = 0;
    // dst = relu(srcs[0] (+ srcs[1])), then dst = relu(dst + srcs[q])
    auto chain = [&](const float *const *srcs, int32_t n, float *dst) -> int {
        {
            acs_args_join a = {dst, srcs[0], n > 1 ? srcs[1] : nullptr, n_act};
            const acs_seg r[2] = {seg(srcs[0], act), seg(n > 1 ? srcs[1] : nullptr, n > 1 ? act : 0)};
            const acs_seg wr[1] = {seg(dst, act)};
            if (int rc = acs_submit(w, ACS_K_JOIN, r, n > 1 ? 2 : 1, wr, 1, &a, sizeof(a), nullptr)) return rc;
            kernels++;
        }
        for (int32_t q = 2; q < n; q++) {
            acs_args_join a = {dst, dst, srcs[q], n_act};
            const acs_seg r[2] = {seg(dst, act), seg(srcs[q], act)};
            const acs_seg wr[1] = {seg(dst, act)};
            if (int rc = acs_submit(w, ACS_K_JOIN, r, 2, wr, 1, &a, sizeof(a), nullptr)) return rc;
            kernels++;
        }
        return ACS_OK;
    };
    // the whole graph is checked before anything is submitted
    if (g->c % 32 != 0 || (g->h * g->h) % 64 != 0) return ACS_EINVAL;
    bool read_by_later[ACS_DAG_MAX_NODES] = {};
    for (int32_t i = 0; i < g->n_nodes; i++) {
        const acs_dag_node &nd = g->node[i];
        if (nd.n_in < 0 || nd.n_in > ACS_DAG_MAX_IN || !nd.w || !nd.b || !nd.y || (nd.n_in > 0 && !nd.agg))
            return ACS_EINVAL;
        for (int32_t q = 0; q < nd.n_in; q++) {
            if (nd.in[q] < 0 || nd.in[q] >= i) return ACS_EINVAL;
            read_by_later[nd.in[q]] = true;
        }
    }
    for (int32_t i = 0; i < g->n_nodes; i++) {
        const acs_dag_node &nd = g->node[i];
        const float *srcs[ACS_DAG_MAX_IN];
        for (int32_t q = 0; q < nd.n_in; q++) srcs[q] = g->node[nd.in[q]].y;
        const float *src = g->x;
        if (nd.n_in > 0) {
            if (int rc = chain(srcs, nd.n_in, nd.agg)) return rc;
            src = nd.agg;
        }
        acs_args_conv a = {src, nd.w, nd.b, nd.y, g->h, g->c, g->c, 3, 1};
        const acs_seg r[3] = {seg(src, act), seg(nd.w, 36ull * g->c * g->c), seg(nd.b, 4ull * g->c)};
        const acs_seg wr[1] = {seg(nd.y, act)};
        if (int rc = acs_submit(w, ACS_K_CONV, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    const float *sinks[ACS_DAG_MAX_NODES];
    int32_t ns = 0;
    for (int32_t i = 0; i < g->n_nodes; i++)
        if (!read_by_later[i]) sinks[ns++] = g->node[i].y;
    if (int rc = chain(sinks, ns, g->sink)) return rc;
    {
        acs_args_avgpool a = {g->pool, g->sink, g->h * g->h, g->c};
        const acs_seg r[1] = {seg(g->sink, act)};
        const acs_seg wr[1] = {seg(g->pool, 4ull * g->c)};
        if (int rc = acs_submit(w, ACS_K_AVGPOOL, r, 1, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    {
        acs_args_fc a = {g->out, g->pool, g->fc_w, g->fc_b, g->c, g->classes};
        const acs_seg r[3] = {seg(g->pool, 4ull * g->c), seg(g->fc_w, 4ull * g->c * g->classes),
                              seg(g->fc_b, 4ull * g->classes)};
        const acs_seg wr[1] = {seg(g->out, 4ull * g->classes)};
        if (int rc = acs_submit(w, ACS_K_FC, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    if (n_kernels) *n_kernels = kernels;
    return ACS_OK;
}

}  // extern "C"

namespace acs {

int dnn_submit_group(acs_window *w, int32_t group, const acs_dnn_graph *g, const float *logits, uint64_t *n_kernels)
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
            if (int rc = acs_submit_group(w, group, ACS_K_CONV, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
            parts[np++] = L.t3;
            kernels++;
        }
        if (g1) {
            acs_args_conv a = {cur, L.w1, L.b1, L.t1, L.hin, L.cin, L.cout, 1, L.stride};
            const acs_seg r[3] = {seg(cur, cur_bytes), seg(L.w1, 4ull * L.cin * L.cout), seg(L.b1, 4ull * L.cout)};
            const acs_seg wr[1] = {seg(L.t1, out_bytes)};
            if (int rc = acs_submit_group(w, group, ACS_K_CONV, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
            parts[np++] = L.t1;
            kernels++;
        }
        if (np > 0) {
            acs_args_join a = {L.y, parts[0], np > 1 ? parts[1] : nullptr, (uint32_t)(out_bytes / 4)};
            const acs_seg r[2] = {seg(parts[0], out_bytes), seg(np > 1 ? parts[1] : nullptr, np > 1 ? out_bytes : 0)};
            const acs_seg wr[1] = {seg(L.y, out_bytes)};
            if (int rc = acs_submit_group(w, group, ACS_K_JOIN, r, np, wr, 1, &a, sizeof(a), nullptr)) return rc;
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
        if (int rc = acs_submit_group(w, group, ACS_K_AVGPOOL, r, 1, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    {
        acs_args_fc a = {g->out, g->pool, g->fc_w, g->fc_b, cur_c, g->classes};
        const acs_seg r[3] = {seg(g->pool, 4ull * cur_c), seg(g->fc_w, 4ull * cur_c * g->classes),
                              seg(g->fc_b, 4ull * g->classes)};
        const acs_seg wr[1] = {seg(g->out, 4ull * g->classes)};
        if (int rc = acs_submit_group(w, group, ACS_K_FC, r, 3, wr, 1, &a, sizeof(a), nullptr)) return rc;
        kernels++;
    }
    if (n_kernels) *n_kernels = kernels;
    return ACS_OK;
}

uint64_t dnn_activation_bytes(const acs_dnn_graph *g)
{
    uint64_t total = 0;
    for (int32_t c = 0; c < g->n_cells; c++) {
        const acs_dnn_cell &L = g->cell[c];
        const uint64_t hout = (uint64_t)(L.hin / (L.stride > 0 ? L.stride : 1));
        total += 3 * rl_align(4 * hout * hout * (uint64_t)L.cout);
    }
    return total + rl_align(4ull * (uint64_t)g->cell[g->n_cells - 1].cout);
}

}  // namespace acs
