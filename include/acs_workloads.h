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
 * buffer, the serving loop's signal words).  NULL on failure.  Free with
 * acs_host_free.  Call neither while a device-path window is open: the HIP
 * host allocator synchronises the whole device, which never completes while
 * the window's scheduler kernel is resident. */
void *acs_host_alloc(size_t bytes);
int acs_host_free(void *p);

/* One rigid-body RL scene.  arena: device memory of acs_rl_layout(n)[ACS_RL_END]
 * bytes with X and V initialised (float4 per body); plan: acs_host_alloc'd
 * int32 buffer of 4 + 4 * (n / 2) entries. */
typedef struct {
    int32_t n;
    int32_t iters;          /* Jacobi iterations per step (8); even (sweeps alternate between Q0 and
                               Q1 and integrate reads Q0), else ACS_EINVAL */
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
 * submitted, the host waits until the islands kernel's plan (the
 * input-dependent island list) carries this step's stamp, while the window
 * keeps running, then iters x (multi-body islands) Jacobi kernels in
 * iteration-major order and the integrate kernel are submitted.  step_ns (if
 * not NULL, `steps` entries) receives the wall time of each step measured
 * between consecutive plan reads; counts (if not NULL) the work done.
 * Returns the first error. */
int acs_rl_run(acs_window *w, const acs_rl_scene *scene, int32_t steps, double *step_ns, acs_rl_counts *counts);

/* Batched scenes (many independent input-dependent graphs in one launch):
 * n_scenes scenes with disjoint arenas, scene i in window group i % n_groups
 * (the window must have acs_config.n_groups >= n_groups; use 1 on paths
 * without groups).  Per batched step: the predicts of every scene are
 * submitted, then every broadphase, every islands and every permute kernel;
 * then, group by group, the host waits for its scenes' plans (their stamps;
 * the window keeps running), reads them and submits their Jacobi kernels
 * iteration by iteration and, within an iteration, island by island across
 * the group's scenes (the k-th island of every scene that has one before any
 * k+1-th), then their integrate kernels.  Each scene's own kernels keep their
 * program order; scenes are independent, so the interleaving changes no
 * result.  step_ns (if not NULL, `steps` entries) receives the wall time
 * of each batched step, which then ends with a full drain; counts the work
 * summed over scenes. */
int acs_rl_run_batch(acs_window *w, const acs_rl_scene *scenes, int32_t n_scenes, int32_t n_groups, int32_t steps,
                     double *step_ns, acs_rl_counts *counts);

/* The graph-per-input baseline (a DAG framework used on an input-dependent
 * graph, Section II-D and Section VI-A): every step's two halves are
 * recorded, built into a HIP graph with their conflict edges (acs_graph_end),
 * launched, waited for and destroyed; the plan is read between them.  Runs
 * on HIP device `device` without a window.  step_ns and counts as for
 * acs_rl_run; build_ns (if not NULL) receives the total time spent
 * recording, building and instantiating the graphs. */
int acs_rl_run_graphs(const acs_rl_scene *scene, int32_t steps, int32_t device, double *step_ns,
                      acs_rl_counts *counts, double *build_ns);

/* Overhead probe: n no-op kernels, each spinning spin_ns on the device.
 * chain = 0: all independent (distinct one-byte write ranges);
 * chain = 1: each reads and writes the same byte (a serial chain).
 * Drains the window at the end; wall_ns receives submit-to-drain time. */
int acs_nop_run(acs_window *w, int32_t n, int32_t chain, uint64_t spin_ns, double *wall_ns);

/* Overhead probe with wider kernels: n independent no-op kernels of nsegs
 * segments each (the first half reads, the rest writes, all disjoint from
 * every other kernel's, each kernel's spread so that its bounding interval
 * meets every other kernel's), so that every dependency check compares
 * nsegs ranges per kernel and finds nothing.  nsegs in [1, 64] (beyond ACS_K_MAX
 * merged as usual).  Drains the window; wall_ns as for acs_nop_run. */
int acs_nop_segs_run(acs_window *w, int32_t n, int32_t nsegs, double *wall_ns);

/* Cost of the host's dependency check (the table of Section IV-D measures
 * the check for W = 16, 32 and 6, 10 read/write segments).  On a manual
 * window of W slots, W - 1 kernels of nsegs disjoint segments each are kept
 * in the window; then reps times a new kernel of nsegs segments, disjoint
 * from all of them, is submitted (checked against the W - 1: every pair of
 * segments is tested), taken and completed.  The same loop with an empty
 * window gives the cost of everything but the check.  Each kernel's segments
 * are spread so that its bounding interval meets every other kernel's: the
 * host's filter on those intervals passes every kernel to the full test.
 * Segments beyond ACS_K_MAX are merged as acs_submit always does
 * (conservative).
 * ns_checked / ns_empty receive nanoseconds per submit-take-complete round
 * with the full and the empty window; tests_out (may be NULL) the segment
 * pairs tested per check.  No GPU is used.  ACS_EINVAL for W outside
 * [2, 64], nsegs outside [2, 64] or reps < 1. */
int acs_check_probe(int32_t W, int32_t nsegs, int32_t reps, double *ns_checked, double *ns_empty, double *tests_out);

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

/* Static irregular network, batch 1 (the static-network workload of Section
 * VI-C; randomly wired): nodes in topological order, all activations
 * h x h x c FP32 NHWC.  A node with no predecessor convolves the input x; a
 * node with predecessors p0, p1, ... first aggregates them into its agg
 * buffer, agg = relu(y[p0] (+ y[p1])), then agg = relu(agg + y[pq]) for
 * q >= 2 (one join kernel each), and convolves agg.  Every convolution is
 * 3x3, stride 1, pad 1, with bias, c -> c.  The nodes no other node reads are
 * aggregated the same way into sink, followed by an average pool and the
 * fully connected head. */
#define ACS_DAG_MAX_NODES 64
#define ACS_DAG_MAX_IN 8
typedef struct {
    int32_t n_in;                     /* 0..ACS_DAG_MAX_IN */
    int32_t in[ACS_DAG_MAX_IN];       /* earlier node indices */
    const float *w, *b;               /* w[3][3][c][c], b[c] */
    float *agg, *y;                   /* [h][h][c] each (agg unused when n_in == 0) */
} acs_dag_node;
typedef struct {
    int32_t n_nodes;                  /* 1..ACS_DAG_MAX_NODES */
    int32_t h, c, classes;
    const float *x;                   /* [h][h][c] */
    acs_dag_node node[ACS_DAG_MAX_NODES];
    float *sink, *pool;               /* [h][h][c], [c] */
    const float *fc_w, *fc_b;         /* [c][classes], [classes] */
    float *out;                       /* [classes] */
} acs_dag_graph;

/* Submits one inference in program order (no drain); *n_kernels (if not
 * NULL) receives the number of kernels.  ACS_EINVAL for a malformed graph
 * (a predecessor that is not an earlier node, shapes the convolution does
 * not take). */
int acs_dag_submit(acs_window *w, const acs_dag_graph *g, uint64_t *n_kernels);

/* Working-memory pool: a host-side allocator over a caller-owned device
 * range [base, base + bytes) (the serving loop's admission budget).  Blocks
 * are 256-byte aligned and sized; best fit, freed blocks merge with free
 * neighbours.  The pool only hands out addresses: it never touches the
 * memory.  acs_pool_create: NULL if base is not 256-byte aligned or bytes <
 * 256.  acs_pool_alloc: ACS_EINVAL for 0 bytes, ACS_ENOMEM when no free block
 * is large enough.  acs_pool_free: ACS_EINVAL for an address that is not a
 * live block.  acs_pool_info: bytes in live blocks, largest free block, live
 * block count (any pointer may be NULL). */
typedef struct acs_pool acs_pool;
acs_pool *acs_pool_create(uint64_t base, uint64_t bytes);
int acs_pool_alloc(acs_pool *p, uint64_t bytes, uint64_t *addr);
int acs_pool_free(acs_pool *p, uint64_t addr);
int acs_pool_info(const acs_pool *p, uint64_t *used, uint64_t *largest_free, int64_t *n_blocks);
void acs_pool_destroy(acs_pool *p);

/* Serving: requests (each one task graph) arrive over time and run
 * concurrently through one window that stays open for the whole run
 * (on the device path: one persistent kernel, window state in device memory).
 *
 * A request is admitted in arrival order (no bypass) once fewer than
 * max_resident requests are in flight and the pool has a block for its
 * working memory; it is then submitted to the window group with the fewest
 * requests in flight.  An RL request is one step of a scene: its input
 * image is copied into its block, predict / broadphase / islands / permute
 * run, and a signal kernel tells the host that the islands kernel has
 * completed; once the plan's stamp is also there the host submits the plan's
 * Jacobi kernels, integrate, a copy of the
 * result out of the block and a final signal.  A DNN request is one
 * inference (acs_dnn_submit's kernels with activations in its block) and a
 * final signal.  The final signal reads the whole block and the output, so
 * it runs after every kernel of the request that wrote them; when the host
 * sees it, the block and the request's slot are released.  Memory reuse
 * between requests is ordered by the window's own range checks within a
 * group, and by the final signal across groups.  Latency is the host time
 * of the final signal minus the arrival time (an open-loop load: a request
 * arrives at its time whether or not the server keeps up). */
enum { ACS_SERVE_RL = 0, ACS_SERVE_DNN = 1 };
typedef struct {
    int32_t kind;              /* ACS_SERVE_RL or ACS_SERVE_DNN */
    int32_t n;                 /* RL: bodies, 2..1024 */
    int32_t iters;             /* RL: Jacobi iterations, even (as in acs_rl_scene) */
    float r, dt;               /* RL: radius, time step */
    int32_t pad;
    double arrival_ns;         /* after the start of the run; non-decreasing over the array */
    uint64_t input;            /* RL: device image of a scene arena's first bytes, X and V at their
                                * acs_rl_layout offsets (off[ACS_RL_V] + 16 n bytes); DNN: x */
    uint64_t output;           /* RL: same layout, X and V after the step; DNN: logits [classes] */
    const float *logits;       /* DNN: host gate logits, 2 per cell; RL: unused */
} acs_serve_request;

typedef struct {
    double admit_ns;           /* first kernel submitted */
    double done_ns;            /* final signal seen by the host */
    uint64_t kernels;          /* kernels submitted, signals and copies included */
    uint64_t footprint;        /* pool bytes held */
    int32_t group;
    int32_t multi_islands;     /* RL: multi-body islands of the step; DNN: -1 */
} acs_serve_result;

typedef struct {
    uint64_t pool, pool_bytes;    /* device range for request working memory (256-byte aligned) */
    void *host;                   /* acs_host_alloc'd, at least acs_serve_host_bytes(max_resident)
                                   * bytes: signal words and island plans, one slot per request in
                                   * flight (allocate it before opening the window) */
    uint64_t host_bytes;
    int32_t max_resident;         /* requests in flight at most, 1..1024 */
    int32_t pad;
    const acs_dnn_graph *model;   /* shapes, weights and head of the network; its
                                   * x, t3, t1, y, pool and out are ignored (NULL if no DNN request) */
    uint64_t stall_ns;            /* ACS_ETIMEDOUT when requests are in flight and none has made
                                   * progress for this long (0: 60 s) */
} acs_serve_config;

typedef struct {
    double wall_ns;               /* start of the run to the last completion */
    uint64_t kernels;
    uint64_t peak_resident;
    uint64_t peak_pool_bytes;
    uint64_t waited_memory;       /* requests that waited at the head of the queue for pool memory */
    uint64_t waited_resident;     /* ... for a free request slot */
} acs_serve_stats;

/* Bytes of host memory acs_serve_run needs for max_resident slots. */
uint64_t acs_serve_host_bytes(int32_t max_resident);

/* Runs n_req requests through window w and drains it.  res (n_req entries)
 * and stats may be NULL.  ACS_EINVAL for bad arguments (a request whose
 * working memory exceeds the whole pool, arrivals out of order, DNN requests
 * without a model, host memory missing or too small); ACS_ETIMEDOUT on a
 * stall; otherwise the window's first error.  It allocates no device or
 * pinned host memory. */
int acs_serve_run(acs_window *w, const acs_serve_config *cfg, const acs_serve_request *req, int32_t n_req,
                  acs_serve_result *res, acs_serve_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* ACS_WORKLOADS_H */
