/*
 * CPU oracle for the windowed out-of-order kernel scheduler (ACS, arXiv 2401.12377).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may include,
 * link or call this code; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes (all plain loops, no blocking, no reordering):
 *   - the byte-range overlap test of Algorithm 1 and the kernel-pair conflict
 *     relation built from it (Section III-C, "Determining inter-kernel
 *     dependencies"; Section IV-B, Algorithm 1);
 *   - the all-pairs dependency DAG of a kernel stream;
 *   - a checker that validates a scheduler trace against that DAG (window
 *     admission, upstream lists, dispatch order, execution intervals);
 *   - in-order (program order) execution of the synthetic workloads' task
 *     bodies, which is by definition the result the scheduler must reproduce
 *     (Section III: the window only reorders kernels it has proven independent).
 */
#ifndef ACS_ORACLE_H
#define ACS_ORACLE_H
#include <stdint.h>

#define OR_KMAX 16

typedef struct { uint64_t start, size; } or_seg;

typedef struct {
    int32_t n_r, n_w;
    or_seg r[OR_KMAX];
    or_seg w[OR_KMAX];
} or_access;

/* Algorithm 1's overlap test on half-open byte ranges; zero-size ranges never overlap. */
int or_overlap(uint64_t s1, uint64_t z1, uint64_t s2, uint64_t z2);
/* Symmetric conflict: newer writes vs older reads+writes, and newer reads vs older writes. */
int or_conflict(const or_access *older, const or_access *newer);
/* Algorithm 1 exactly as printed: only the newer kernel's writes vs the older's reads+writes. */
int or_conflict_literal(const or_access *older, const or_access *newer);
/* adj[i*n+j] = 1 iff i < j and kernels i, j conflict. */
void or_dag(int32_t n, const or_access *acc, int32_t literal, uint8_t *adj);

typedef struct {
    int64_t seq, slot, kid;
    int64_t ev_insert, ev_dispatch, ev_retire;
    uint64_t valid_mask;   /* slots occupied by older kernels when this one was inserted */
    uint64_t up_mask;      /* upstream slots recorded at insert */
    int64_t t_start, t_end;/* execution interval on one clock, or -1 when not recorded */
    int64_t t_dispatch, t_retire; /* informational, not checked */
} or_trace_rec;

/* 0 when the trace is a valid schedule of the stream with window W; else a code
 * and a message.  check_times != 0 also checks the execution intervals.
 * early != 0 accepts a kernel handed out before its upstream kernels retired,
 * provided they were handed out before it and (times then required) its
 * execution interval starts after theirs end. */
int32_t or_check_trace(int32_t n, const or_access *acc, int32_t W, const or_trace_rec *tr,
                       int32_t check_times, int32_t early, char *msg, int32_t msglen);

/* ---------------- tiny random stream ---------------- */
enum { OR_OP_SCALE = 0, OR_OP_AXPY = 1, OR_OP_SUM = 2 };
typedef struct { int32_t op, out, nin, in[3], j; float a; } or_tiny_kernel;

void or_tiny_access(const int64_t *offs, const int64_t *lens, uint64_t base,
                    const or_tiny_kernel *k, or_access *acc);
/* Runs the kernels in `order` (NULL = program order) on the arena (floats). */
void or_tiny_run(float *arena, const int64_t *offs, const int64_t *lens,
                 int32_t nk, const or_tiny_kernel *ks, const int32_t *order);
float or_tree_sum(const float *v, int64_t n);

/* ---------------- rigid-body RL step ---------------- */
typedef struct {
    int32_t n, iters;
    float r, dt;
    float *X, *V, *P, *Q0, *Q1;              /* 4 floats per body */
    int32_t *deg, *adj_off, *adj;            /* n, n+1, n*(n-1) */
    int32_t *label, *perm, *inv_perm, *isl_off;   /* n, n, n, n+1 */
    int32_t *padj_off, *padj;                /* n+1, n*(n-1) */
    int32_t *meta;                           /* [0]=islands, [1]=multi-body islands, [2]=directed edges */
    int32_t *plan;                           /* 4 per multi-body island: pos begin/end, edge begin/end */
} or_scene;

enum { OR_RL_PREDICT = 0, OR_RL_BROADPHASE, OR_RL_ISLANDS, OR_RL_PERMUTE, OR_RL_JACOBI, OR_RL_INTEGRATE };
typedef struct { int32_t op, island, iter; } or_rl_kernel;

void or_rl_run_kernel(or_scene *s, const or_rl_kernel *k);
void or_rl_access(const or_scene *s, const or_rl_kernel *k, or_access *acc);
/* Kernel list of one step in program order; the Jacobi part needs the plan,
 * so call after the islands kernel has run.  Returns the count written. */
int32_t or_rl_step_kernels(const or_scene *s, or_rl_kernel *out, int32_t cap);
/* One whole step in program order. */
void or_rl_step(or_scene *s);

/* ---------------- dynamic DNN (batch 1, NHWC) ----------------
 * The dynamic-network case study (Section II-C): convolutions whose execution
 * is decided per input.  Tensors are NHWC with batch 1: act[y][x][c].
 *
 * Convolution with kernel k in {1, 3} (3x3 zero-padded by 1) and stride s:
 *   out[y][x][co] = bias[co] + sum over (ky, kx, ci) of
 *                   in[y*s + ky - p][x*s + kx - p][ci] * w[ky][kx][ci][co]
 * with p = (k - 1) / 2 and hout = (hin + 2p - k) / s + 1.
 * or_conv_f32: FP32, the products accumulated with fmaf from 0 in
 *   (ky, kx, ci) order, the bias added last (one defined order).
 * or_conv_f64: the same sum in double, and mag = the sum of the absolute
 *   values of its terms (|bias| included), for error bounds. */
int32_t or_conv_hout(int32_t hin, int32_t k, int32_t s);
void or_conv_f32(const float *in, const float *w, const float *b, float *out,
                 int32_t hin, int32_t cin, int32_t cout, int32_t k, int32_t s);
void or_conv_f64(const float *in, const float *w, const float *b, double *out, double *mag,
                 int32_t hin, int32_t cin, int32_t cout, int32_t k, int32_t s);
/* relu(x) = x if x > 0 else +0 (so -0 and NaN give +0) */
float or_relu(float x);
/* out = relu(a + b) elementwise, or relu(a) when b is NULL */
void or_join(float *out, const float *a, const float *b, int64_t n);
/* out[c] = (sum over the hw pixels, in pixel order, in FP32) / hw */
void or_avgpool(float *out, const float *in, int32_t hw, int32_t c);
/* out[j] = b[j] + sum_i in[i] * w[i][j]: acc = b[j], then acc = fmaf(in[i], w[i][j], acc) for i = 0.. */
void or_fc(float *out, const float *in, const float *w, const float *b, int32_t cin, int32_t cout);

#endif
