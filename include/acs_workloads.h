/*
 * acs_workloads.h - native drivers that play the application on top of the
 * acs.h API for the synthetic workloads (the paper's evaluation runs
 * physics-simulation steps whose kernel graph depends on the input,
 * Section II-B and Section VI).  They only call acs_submit / acs_sync and
 * read results; they hold no scheduling logic of their own.
 */
#ifndef ACS_WORKLOADS_H
#define ACS_WORKLOADS_H

#include <stddef.h>
#include <stdint.h>

#include "acs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Pinned, coherent host memory that kernels can write directly (the RL plan
 * buffer).  NULL on failure.  Free with acs_host_free. */
void *acs_host_alloc(size_t bytes);
int acs_host_free(void *p);

/* One rigid-body RL scene.  arena: device memory of acs_rl_layout(n)[ACS_RL_END]
 * bytes with X and V initialised (float4 per body); plan: acs_host_alloc'd
 * int32 buffer of 4 + 4 * (n / 2) entries. */
typedef struct {
    int32_t n;
    int32_t iters;          /* Jacobi iterations per step (8) */
    float r, dt;
    uint64_t arena;
    int32_t *plan;
} acs_rl_scene;

/* Work done by acs_rl_run, summed over its steps. */
typedef struct {
    uint64_t kernels;          /* kernels submitted */
    uint64_t steps;
    uint64_t islands;          /* connected components found */
    uint64_t multi_islands;    /* components with two or more bodies */
    uint64_t edges;            /* directed contact edges (twice the contacts) */
    uint64_t jacobi_kernels;
    uint64_t jacobi_bodies;    /* bodies covered by Jacobi kernels */
    uint64_t jacobi_edges;     /* adjacency entries read by Jacobi kernels */
} acs_rl_counts;

/* Runs `steps` steps.  Per step: predict, broadphase, islands, permute are
 * submitted, the window is drained so that the plan (input-dependent island
 * list) can be read, then iters x (multi-body islands) Jacobi kernels in
 * iteration-major order and the integrate kernel are submitted.  step_ns (if
 * not NULL, `steps` entries) receives the wall time of each step measured
 * between consecutive plan reads; counts (if not NULL) the work done.
 * Returns the first error. */
int acs_rl_run(acs_window *w, const acs_rl_scene *scene, int32_t steps, double *step_ns, acs_rl_counts *counts);

/* Batched scenes (many independent input-dependent graphs in one launch):
 * n_scenes scenes with disjoint arenas, scene i in window group i % n_groups
 * (the window must have acs_config.n_groups >= n_groups; use 1 on paths
 * without groups).  Per batched step: every scene's predict, broadphase,
 * islands and permute are submitted; then, group by group, the group is
 * drained, its scenes' plans read and their Jacobi and integrate kernels
 * submitted.  step_ns (if not NULL, `steps` entries) receives the wall time
 * of each batched step, which then ends with a full drain; counts the work
 * summed over scenes. */
int acs_rl_run_batch(acs_window *w, const acs_rl_scene *scenes, int32_t n_scenes, int32_t n_groups, int32_t steps,
                     double *step_ns, acs_rl_counts *counts);

/* Overhead probe: n no-op kernels, each spinning spin_ns on the device.
 * chain = 0: all independent (distinct one-byte write ranges);
 * chain = 1: each reads and writes the same byte (a serial chain).
 * Drains the window at the end; wall_ns receives submit-to-drain time. */
int acs_nop_run(acs_window *w, int32_t n, int32_t chain, uint64_t spin_ns, double *wall_ns);

/* Dynamic DNN, batch 1 (the dynamic-network case study, Section II-C): cells
 * of two parallel gated branches, a 3x3 (pad 1) and a 1x1 convolution with
 * the cell's stride, joined by relu(sum of the branches that ran); a cell
 * with no branch is the identity.  Then an average pool and a fully connected
 * head.  All tensors are FP32 NHWC device buffers owned by the caller. */
#define ACS_DNN_MAX_CELLS 16
typedef struct {
    int32_t hin, cin, cout, stride;   /* stride 1 or 2; hout = hin / stride */
    const float *w3, *b3;             /* w3[3][3][cin][cout], b3[cout] */
    const float *w1, *b1;             /* w1[cin][cout], b1[cout] */
    float *t3, *t1, *y;               /* [hout][hout][cout]: 3x3 branch, 1x1 branch, cell output */
} acs_dnn_cell;
typedef struct {
    int32_t n_cells;                  /* 1..ACS_DNN_MAX_CELLS */
    int32_t classes;
    const float *x;                   /* input [hin][hin][cin] of cell 0 */
    acs_dnn_cell cell[ACS_DNN_MAX_CELLS];
    float *pool;                      /* [cout of the last cell] */
    const float *fc_w, *fc_b;         /* [cout_last][classes], [classes] */
    float *out;                       /* [classes] */
} acs_dnn_graph;

/* Submits one inference in program order (no drain).  Per cell c: the 3x3
 * branch if logits[2c] > 0; the 1x1 branch if logits[2c+1] > 0 or the cell
 * has stride 2 (so that a cell that changes shape always has an output); the
 * join if either ran, reading the previous cell output that exists (or x).
 * Then average pool and the head.  Each kernel's ranges are its whole input
 * and output tensors and its weights.  *n_kernels (if not NULL) receives the
 * number of kernels submitted.  Returns 0 or the first error. */
int acs_dnn_submit(acs_window *w, const acs_dnn_graph *g, const float *logits, uint64_t *n_kernels);

#ifdef __cplusplus
}
#endif
#endif /* ACS_WORKLOADS_H */
