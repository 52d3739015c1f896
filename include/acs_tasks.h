/*
 * acs_tasks.h - the closed table of task bodies the library can run, and the
 * argument struct of each.  A kernel_id passed to acs_submit names one of
 * these; its args block is the matching struct (at most ACS_ARGS_MAX bytes).
 *
 * The paper's kernel wrapper pairs a kernel with a function that states its
 * read and write ranges from its launch arguments (Section IV-A).  Here the
 * body is chosen from this table and the caller states the ranges; the
 * Python binding has one range helper per task type.
 *
 * Every body runs with 256-thread workgroups.  A splittable body is cut into
 * "pieces" (one workgroup each); its result never depends on the number of
 * pieces, so all paths produce identical bits.
 */
#ifndef ACS_TASKS_H
#define ACS_TASKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum acs_kernel_id {
    ACS_K_NOP = 0,            /* empty body, optional busy wait (overhead measurements) */
    /* tiny random stream */
    ACS_K_SCALE = 1,          /* out[i] = a * x[i],            i < n */
    ACS_K_AXPY = 2,           /* out[i] = fma(a, x[i], y[i]),  i < n */
    ACS_K_SUM = 3,            /* *out = pairwise sum of in[0..nin) concatenated */
    /* rigid-body RL step (one scene; see acs_rl_layout) */
    ACS_K_RL_PREDICT = 10,    /* P = fma(dt, V, X) */
    ACS_K_RL_BROADPHASE = 11, /* all-pairs contact test on P -> degree + adjacency (CSR) */
    ACS_K_RL_ISLANDS = 12,    /* connected components -> permutation, permuted CSR, plan */
    ACS_K_RL_PERMUTE = 13,    /* Q0[p] = P[perm[p]] */
    ACS_K_RL_JACOBI = 14,     /* one Jacobi contact iteration over one island */
    ACS_K_RL_INTEGRATE = 15,  /* X, V from Q0 with wall reflection */
    /* dynamic DNN, batch 1, NHWC FP32 (acs_args_conv etc.) */
    ACS_K_CONV = 20,          /* 3x3 (pad 1) or 1x1 convolution, stride 1 or 2, + bias; FP32 MFMA */
    ACS_K_JOIN = 21,          /* out = relu(a + b), or relu(a) when b is NULL */
    ACS_K_AVGPOOL = 22,       /* out[c] = (sum of in[q][c] over the hw pixels, in pixel order) / hw */
    ACS_K_FC = 23,            /* out[j] = b[j] + sum_i in[i] w[i][j], fmaf chain in i order */
    /* request plumbing (serving) */
    ACS_K_COPY = 24,          /* dst[0..bytes) = src[0..bytes), bit copy */
    ACS_K_SIGNAL = 25,        /* *addr = value, a release store visible to the host */
    ACS_K_COUNT = 26
};

#define ACS_BLOCK 256

typedef struct { uint64_t spin_ns; } acs_args_nop;

typedef struct { float *out; const float *x; float a; uint32_t n; } acs_args_scale;

typedef struct { float *out; const float *x; const float *y; float a; uint32_t n; } acs_args_axpy;

/* in[k] holds len[k] floats; the sum runs over in[0] ++ in[1] ++ ... (nin <= 3).
 * Pairwise tree: pad with zeros to the next power of two P and, for
 * s = P/2, ..., 1, add element i + s into element i. */
typedef struct { float *out; const float *in[3]; uint32_t len[3]; uint32_t nin; } acs_args_sum;

/* Rigid-body RL scene.  `base` is the scene's device arena (acs_rl_layout);
 * `plan` is a host-visible int32 buffer of 4 + 4 * (n / 2) entries written by
 * the islands kernel: [0] islands, [1] multi-body islands, [2] directed edges,
 * [3] the islands kernel's `iter` argument (a stamp), then per multi-body
 * island: first position, end position, first edge, end edge.  Every entry
 * is a system-scope store and the stamp is stored after all the others have
 * completed, so a host that sees its stamp in [3] (acquire load) may read the
 * plan while the window is still running.  Only the host reads the plan: on
 * the device-resident path it is stored after the islands kernel has been
 * marked complete (its dependents do not wait for host memory), so the
 * kernel's completion alone does not make the plan readable; the stamp
 * does. */
typedef struct {
    uint64_t base;
    uint64_t plan;
    int32_t n;
    float r;
    float dt;
    int32_t iter;            /* Jacobi: iteration index (even: Q0 -> Q1, odd: Q1 -> Q0);
                                islands: the stamp stored last into plan[3] */
    int32_t b0, b1;          /* Jacobi: positions [b0, b1) of the island */
} acs_args_rl;

/* Convolution over an NHWC activation in[hin][hin][cin] with weights
 * w[k][k][cin][cout] (k = 1: w[cin][cout]) and bias[cout], into
 * out[hout][hout][cout], hout = (hin + 2p - k) / stride + 1, p = (k - 1) / 2.
 * Implicit GEMM M = hout^2, N = cout, K = k^2 cin on 16x16x4 FP32 MFMA tiles;
 * requires cin % 32 == 0, cout % 32 == 0, hout^2 % 16 == 0.  Sums are FP32
 * in the matrix unit's order (not the scalar reference's): checked against a
 * float64 reference within 1e-5 of the sum of |terms|.  One piece per 16 x 32
 * output tile; the four waves of a piece split K and add their partial tiles
 * in wave order. */
typedef struct {
    const float *in;
    const float *w;
    const float *bias;
    float *out;
    int32_t hin, cin, cout, k, stride;
} acs_args_conv;
typedef struct { float *out; const float *a; const float *b; uint32_t n; } acs_args_join;
typedef struct { float *out; const float *in; int32_t hw, c; } acs_args_avgpool;
typedef struct { float *out; const float *in; const float *w; const float *bias; int32_t cin, cout; } acs_args_fc;

/* Bit copy of `bytes` bytes; dst and src 16-byte aligned, bytes a multiple
 * of 16, the two ranges disjoint.  Used to stage a request's input into its
 * working memory and its result out of it. */
typedef struct { void *dst; const void *src; uint64_t bytes; } acs_args_copy;

/* Stores `value` into the 8-byte word at addr (host-visible memory allowed)
 * with release ordering at system scope: every write of a kernel this one
 * depended on is visible before the value is.  Its read ranges state what
 * it waits for; its write range is the word.  One workgroup. */
typedef struct { uint64_t *addr; uint64_t value; } acs_args_signal;

/* Regions of an RL scene arena, in order; byte offsets from acs_rl_layout. */
enum acs_rl_region {
    ACS_RL_X = 0, ACS_RL_V, ACS_RL_P, ACS_RL_Q0, ACS_RL_Q1,       /* float4[n] */
    ACS_RL_DEG, ACS_RL_ADJ_OFF, ACS_RL_ADJ,                       /* int[n], int[n+1], int[n(n-1)] */
    ACS_RL_LABEL, ACS_RL_PERM, ACS_RL_INV_PERM, ACS_RL_ISL_OFF,   /* int[n] x3, int[n+1] */
    ACS_RL_PADJ_OFF, ACS_RL_PADJ,                                 /* int[n+1], int[n(n-1)] */
    ACS_RL_END,                                                   /* total arena bytes */
    ACS_RL_NREGIONS
};

/* Fills off[ACS_RL_NREGIONS] with 256-byte-aligned offsets for n bodies;
 * returns 0, or ACS_EINVAL (-1) when n is outside [2, 1024]. */
int acs_rl_layout(int32_t n, uint64_t *off);

#ifdef __cplusplus
}
#endif
#endif /* ACS_TASKS_H */
