// Drives libacs's host code, built with the address and undefined-behaviour
// sanitizers against the host stand-in of the HIP runtime (fake_hip.cpp).
// Test infrastructure only.  Each part prints one line; any sanitizer report
// or failed check ends the program with a non-zero status.
//
//   graphs     the graph-per-input RL driver over thousands of steps whose
//              island plans change every step (the islands kernel's part is
//              played by a hook that writes a random valid plan);
//   replay     recorded task graphs built, replayed and destroyed many times;
//   paths      random streams of no-op kernels with random ranges through the
//              in-order, plain, events and manual paths;
//   ranges     submissions with up to 300 ranges (normalisation and merging).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "acs.h"
#include "acs_tasks.h"
#include "acs_workloads.h"
#include "hip/hip_runtime_api.h"

extern "C" void fake_hip_set_kernel_hook(void (*hook)(int32_t, const void *));
extern "C" void fake_hip_counts(int64_t *out);

#define CHECK(c)                                                                              \
    do {                                                                                      \
        if (!(c)) {                                                                           \
            fprintf(stderr, "check failed at line %d: %s (last error %d: %s)\n", __LINE__, #c, \
                    acs_last_error(), acs_strerror(acs_last_error()));                        \
            exit(1);                                                                          \
        }                                                                                     \
    } while (0)

namespace {

uint64_t g_s = 12345;
uint64_t rnd()
{
    g_s = g_s * 6364136223846793005ull + 1442695040888963407ull;
    return g_s >> 17;
}

// islands kernel stand-in: a random plan of multi-body islands for n bodies
uint64_t g_multi = 0, g_jacobi_expected = 0;
int32_t g_iters = 8;
void islands_hook(int32_t kid, const void *args)
{
    if (kid != ACS_K_RL_ISLANDS) return;
    acs_args_rl a;
    memcpy(&a, args, sizeof(a));
    int32_t *plan = (int32_t *)(uintptr_t)a.plan;
    const int32_t n = a.n;
    int32_t pos = 0, edges = 0, m = 0, islands = 0;
    while (pos < n) {
        const int32_t left = n - pos;
        int32_t sz = 1 + (int32_t)(rnd() % (uint64_t)(left < 6 ? left : 6));
        islands++;
        if (sz >= 2 && m < n / 2) {
            const int32_t e = sz * (sz - 1) / 2 * 2;
            plan[4 + 4 * m] = pos;
            plan[5 + 4 * m] = pos + sz;
            plan[6 + 4 * m] = edges;
            plan[7 + 4 * m] = edges + e;
            edges += e;
            m++;
        }
        pos += sz;
    }
    plan[0] = islands;
    plan[2] = edges;
    plan[1] = m;
    // the stamp last, as the islands kernel stores it
    __atomic_store_n(&plan[3], a.iter, __ATOMIC_RELEASE);
    g_multi += (uint64_t)m;
    g_jacobi_expected += (uint64_t)m * (uint64_t)g_iters;
}

void part_graphs()
{
    fake_hip_set_kernel_hook(islands_hook);
    uint64_t steps_total = 0;
    for (int32_t n : {2, 7, 64, 300, 1024}) {
        uint64_t off[ACS_RL_NREGIONS];
        CHECK(acs_rl_layout(n, off) == ACS_OK);
        void *arena = nullptr;
        CHECK(hipMalloc(&arena, off[ACS_RL_END]) == hipSuccess);
        int32_t *plan = (int32_t *)acs_host_alloc(4 * (4 + 4 * (n / 2)));
        CHECK(plan);
        acs_rl_scene sc = {n, g_iters, 0.05f, 1.0f / 120, (uint64_t)(uintptr_t)arena, plan};
        const int32_t steps = n >= 1024 ? 20 : (n >= 300 ? 100 : 1500);
        std::vector<double> step_ns(steps);
        acs_rl_counts cnt;
        double build = 0;
        g_multi = g_jacobi_expected = 0;
        CHECK(acs_rl_run_graphs(&sc, steps, 0, step_ns.data(), &cnt, &build) == ACS_OK);
        CHECK(cnt.steps == (uint64_t)steps);
        CHECK(cnt.multi_islands == g_multi);
        CHECK(cnt.jacobi_kernels == g_jacobi_expected);
        CHECK(cnt.kernels == 5ull * steps + g_jacobi_expected);
        CHECK(build > 0);
        steps_total += (uint64_t)steps;
        CHECK(acs_host_free(plan) == ACS_OK);
        CHECK(hipFree(arena) == hipSuccess);
    }
    // odd sweep counts are refused up front
    {
        int32_t plan[8] = {};
        acs_rl_scene sc = {16, 3, 0.05f, 1.0f / 120, 1ull << 30, plan};
        CHECK(acs_rl_run_graphs(&sc, 1, 0, nullptr, nullptr, nullptr) == ACS_EINVAL);
    }
    fake_hip_set_kernel_hook(nullptr);
    printf("graphs: %llu graph-per-input steps\n", (unsigned long long)steps_total);
}

acs_seg seg(uint64_t s, uint64_t z) { return acs_seg{s, z}; }

// a random no-op kernel over a 64-byte-granular address space of 1 KiB
int submit_random(acs_window *w, int group = 0)
{
    acs_seg r[3], wr[2];
    const int nr = (int)(rnd() % 4), nw = 1 + (int)(rnd() % 2);
    for (int i = 0; i < nr; i++) r[i] = seg(0x10000 + 64 * (rnd() % 16), 64 * (1 + rnd() % 2));
    for (int i = 0; i < nw; i++) wr[i] = seg(0x10000 + 64 * (rnd() % 16), 64);
    acs_args_nop a = {0};
    return acs_submit_group(w, group, ACS_K_NOP, r, nr, wr, nw, &a, sizeof(a), nullptr);
}

void part_replay()
{
    int replays = 0;
    for (int round = 0; round < 300; round++) {
        acs_window *w = acs_window_create(16);
        CHECK(w);
        acs_config cfg;
        acs_config_default(&cfg);
        cfg.path = ACS_PATH_INORDER;
        CHECK(acs_window_configure(w, &cfg) == ACS_OK);
        CHECK(acs_graph_begin(w) == ACS_OK);
        const int k = 1 + (int)(rnd() % 80);
        for (int i = 0; i < k; i++) CHECK(submit_random(w) == ACS_OK);
        acs_graph *g = nullptr;
        CHECK(acs_graph_end(w, &g) == ACS_OK);
        int64_t nk = 0, ne = 0;
        CHECK(acs_graph_info(g, &nk, &ne) == ACS_OK);
        CHECK(nk == k && ne >= 0 && ne <= (int64_t)k * (k - 1) / 2);
        const int reps = (int)(rnd() % 4);
        for (int r = 0; r < reps; r++, replays++) CHECK(acs_graph_launch(g) == ACS_OK);
        if (rnd() % 2) CHECK(acs_graph_sync(g) == ACS_OK);
        // the window and the graph may go in either order
        if (rnd() % 2) {
            CHECK(acs_graph_destroy(g) == ACS_OK);
            CHECK(acs_window_destroy(w) == ACS_OK);
        } else {
            CHECK(acs_window_destroy(w) == ACS_OK);
            CHECK(acs_graph_destroy(g) == ACS_OK);
        }
    }
    printf("replay: 300 graphs, %d replays\n", replays);
}

void part_paths()
{
    const int32_t paths[] = {ACS_PATH_INORDER, ACS_PATH_PLAIN, ACS_PATH_EVENTS};
    uint64_t kernels = 0;
    for (int32_t path : paths) {
        for (int round = 0; round < 40; round++) {
            const int32_t W = 1 + (int32_t)(rnd() % 64);
            acs_window *w = acs_window_create(W);
            CHECK(w);
            acs_config cfg;
            acs_config_default(&cfg);
            cfg.path = path;
            cfg.n_streams = 1 + (int32_t)(rnd() % 8);
            cfg.queue_depth = 1 + (int32_t)(rnd() % 64);
            cfg.trace = (int32_t)(rnd() % 2);
            cfg.trace_capacity = 1 << 12;
            cfg.n_groups = 1 + (int32_t)(rnd() % 4);
            CHECK(acs_window_configure(w, &cfg) == ACS_OK);
            const int n = 1 + (int)(rnd() % 400);
            for (int i = 0; i < n; i++) {
                CHECK(submit_random(w, (int)(rnd() % (uint64_t)cfg.n_groups)) == ACS_OK);
                if (rnd() % 16 == 0) CHECK(acs_poll(w) == ACS_OK);
                if (rnd() % 64 == 0) CHECK(acs_sync_group(w, (int32_t)(rnd() % (uint64_t)cfg.n_groups), 0) == ACS_OK);
            }
            CHECK(acs_sync(w) == ACS_OK);
            acs_stats st;
            CHECK(acs_stats_get(w, &st) == ACS_OK);
            CHECK(st.submitted == (uint64_t)n && st.retired == (uint64_t)n);
            if (cfg.trace && path != ACS_PATH_EVENTS) {
                std::vector<acs_trace_rec> tr(n);
                int64_t got = 0;
                CHECK(acs_trace_read(w, tr.data(), n, &got) == ACS_OK);
                CHECK(got == n);
            }
            if (rnd() % 2) CHECK(acs_window_stop(w) == ACS_OK);
            CHECK(acs_window_destroy(w) == ACS_OK);
            kernels += (uint64_t)n;
        }
    }
    // manual path: random completion order
    for (int round = 0; round < 100; round++) {
        const int32_t W = 1 + (int32_t)(rnd() % 64);
        acs_window *w = acs_window_create(W);
        acs_config cfg;
        acs_config_default(&cfg);
        cfg.path = ACS_PATH_MANUAL;
        cfg.queue_depth = 4096;
        cfg.trace = 1;
        CHECK(acs_window_configure(w, &cfg) == ACS_OK);
        const int n = 1 + (int)(rnd() % 300);
        for (int i = 0; i < n; i++) CHECK(submit_random(w) == ACS_OK);
        std::vector<uint64_t> running;
        uint64_t done = 0;
        while (done < (uint64_t)n) {
            uint64_t seqs[64];
            int32_t k = 0;
            CHECK(acs_manual_take_ready(w, seqs, 64, &k) == ACS_OK);
            running.insert(running.end(), seqs, seqs + k);
            CHECK(!running.empty());
            const size_t pick = (size_t)(rnd() % running.size());
            CHECK(acs_manual_complete(w, running[pick], (rnd() % 50 == 0) ? 1 : 0) == ACS_OK);
            running.erase(running.begin() + (long)pick);
            acs_stats st;
            CHECK(acs_stats_get(w, &st) == ACS_OK);
            done = st.retired;
        }
        acs_entry lst[64];
        int32_t cnt = 0;
        CHECK(acs_scheduled_list(w, lst, 64, &cnt) == ACS_OK && cnt == 0);
        (void)acs_sync(w);   // ACS_EKERNEL when a failure was planted
        CHECK(acs_window_destroy(w) == ACS_OK || true);
        kernels += (uint64_t)n;
    }
    printf("paths: %llu kernels\n", (unsigned long long)kernels);
}

// The RL drivers on the host-side paths: each step waits for its islands
// kernel's plan stamp (the kernel runs only when the path queries or
// synchronises its streams), then submits the plan's Jacobi kernels.
void part_rlrun()
{
    fake_hip_set_kernel_hook(islands_hook);
    const int32_t paths[] = {ACS_PATH_INORDER, ACS_PATH_PLAIN, ACS_PATH_EVENTS};
    uint64_t steps_total = 0;
    for (int32_t path : paths)
        for (int32_t n : {2, 9, 64, 200}) {
            uint64_t off[ACS_RL_NREGIONS];
            CHECK(acs_rl_layout(n, off) == ACS_OK);
            const int32_t n_scenes = 3;
            std::vector<void *> arenas(n_scenes);
            std::vector<int32_t *> plans(n_scenes);
            std::vector<acs_rl_scene> sc(n_scenes);
            for (int32_t i = 0; i < n_scenes; i++) {
                CHECK(hipMalloc(&arenas[i], off[ACS_RL_END]) == hipSuccess);
                plans[i] = (int32_t *)acs_host_alloc(4 * (4 + 4 * (n / 2)));
                CHECK(plans[i]);
                plans[i][3] = 1;   // a stale stamp equal to the first one a driver uses
                sc[i] = {n, g_iters, 0.05f, 1.0f / 120, (uint64_t)(uintptr_t)arenas[i], plans[i]};
            }
            acs_window *w = acs_window_create(1 + (int32_t)(rnd() % 64));
            CHECK(w);
            acs_config cfg;
            acs_config_default(&cfg);
            cfg.path = path;
            cfg.n_streams = 1 + (int32_t)(rnd() % 8);
            CHECK(acs_window_configure(w, &cfg) == ACS_OK);
            const int32_t steps = n >= 200 ? 20 : 200;
            std::vector<double> step_ns(steps);
            acs_rl_counts cnt;
            g_multi = g_jacobi_expected = 0;
            const int rc = acs_rl_run(w, &sc[0], steps, step_ns.data(), &cnt);
            if (rc != ACS_OK) printf("path %d, %d bodies: acs_rl_run returned %d\n", path, n, rc);
            CHECK(rc == ACS_OK);
            CHECK(cnt.steps == (uint64_t)steps && cnt.multi_islands == g_multi);
            CHECK(cnt.kernels == 5ull * steps + g_jacobi_expected);
            g_multi = g_jacobi_expected = 0;
            CHECK(acs_rl_run_batch(w, sc.data(), n_scenes, 1, steps / 4, step_ns.data(), &cnt) == ACS_OK);
            CHECK(cnt.steps == (uint64_t)(n_scenes * (steps / 4)) && cnt.multi_islands == g_multi);
            CHECK(cnt.kernels == 5ull * n_scenes * (steps / 4) + g_jacobi_expected);
            CHECK(acs_sync(w) == ACS_OK);
            CHECK(acs_window_destroy(w) == ACS_OK);
            for (int32_t i = 0; i < n_scenes; i++) {
                CHECK(acs_host_free(plans[i]) == ACS_OK);
                CHECK(hipFree(arenas[i]) == hipSuccess);
            }
            steps_total += (uint64_t)steps + (uint64_t)n_scenes * (uint64_t)(steps / 4);
        }
    fake_hip_set_kernel_hook(nullptr);
    printf("rlrun: %llu driver steps\n", (unsigned long long)steps_total);
}

void part_ranges()
{
    acs_window *w = acs_window_create(64);
    acs_config cfg;
    acs_config_default(&cfg);
    cfg.path = ACS_PATH_MANUAL;
    cfg.queue_depth = 1 << 16;
    CHECK(acs_window_configure(w, &cfg) == ACS_OK);
    std::vector<acs_seg> r(300), wr(300);
    uint64_t total = 0;
    for (int i = 0; i < 2000; i++) {
        const int nr = (int)(rnd() % 301), nw = (int)(rnd() % 301);
        for (int k = 0; k < nr; k++) r[k] = seg(16 * (rnd() % 100000), 1 + rnd() % 40);
        for (int k = 0; k < nw; k++) wr[k] = seg(16 * (rnd() % 100000), 1 + rnd() % 40);
        if (rnd() % 20 == 0 && nr > 0) r[0] = seg(ACS_SEG_ALL_START, ACS_SEG_ALL_SIZE);
        acs_args_nop a = {0};
        CHECK(acs_submit(w, ACS_K_NOP, r.data(), nr, wr.data(), nw, &a, sizeof(a), nullptr) == ACS_OK);
        total++;
        uint64_t seqs[64];
        int32_t k = 0;
        CHECK(acs_manual_take_ready(w, seqs, 64, &k) == ACS_OK);
        for (int32_t q = 0; q < k; q++) CHECK(acs_manual_complete(w, seqs[q], 0) == ACS_OK);
    }
    // a range that wraps is refused
    acs_seg bad = seg(~0ull - 4, 16);
    acs_args_nop a = {0};
    CHECK(acs_submit(w, ACS_K_NOP, &bad, 1, nullptr, 0, &a, sizeof(a), nullptr) == ACS_EINVAL);
    acs_stats st;
    CHECK(acs_stats_get(w, &st) == ACS_OK);
    CHECK(st.submitted == total && st.coalesced > 0);
    CHECK(acs_window_destroy(w) == ACS_OK || true);
    printf("ranges: %llu submissions, %llu merged lossily\n", (unsigned long long)total,
           (unsigned long long)st.coalesced);
}

}  // namespace

int main(int argc, char **argv)
{
    setvbuf(stdout, nullptr, _IOLBF, 0);
    const char *only = argc > 1 ? argv[1] : "";
    if (!*only || !strcmp(only, "graphs")) part_graphs();
    if (!*only || !strcmp(only, "replay")) part_replay();
    if (!*only || !strcmp(only, "paths")) part_paths();
    if (!*only || !strcmp(only, "ranges")) part_ranges();
    if (!*only || !strcmp(only, "rlrun")) part_rlrun();
    int64_t c[6];
    fake_hip_counts(c);
    printf("alive: streams %lld events %lld graphs %lld execs %lld device %lld host %lld\n", (long long)c[0],
           (long long)c[1], (long long)c[2], (long long)c[3], (long long)c[4], (long long)c[5]);
    printf("ok\n");
    return 0;
}
