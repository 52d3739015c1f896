/*
 * CPU oracle for the windowed out-of-order kernel scheduler (ACS, arXiv 2401.12377).
 * TEST INFRASTRUCTURE ONLY: see acs_oracle.h.  Built with -O2 -ffp-contract=off
 * so that every floating-point operation below is exactly the one written.
 *
 * Task-body precision: the paper fixes no arithmetic for task bodies.  The
 * synthetic workloads are defined as FP32 programs with a fixed operation
 * order (explicit fmaf where the definition says fused, a fixed pairwise tree
 * for sums, correctly rounded sqrt and division), so that every integer
 * decision (contacts, islands) is taken in the same precision on both sides.
 */
#include "acs_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Overlap and conflict (Section III-C; Section IV-B, Algorithm 1)                          */
/* ------------------------------------------------------------------------ */

static uint64_t seg_end(uint64_t start, uint64_t size)
{
    /* saturate: {0, UINT64_MAX} stands for "all of memory" (Section IV-A) */
    return (size > UINT64_MAX - start) ? UINT64_MAX : start + size;
}

int or_overlap(uint64_t s1, uint64_t z1, uint64_t s2, uint64_t z2)
{
    if (z1 == 0 || z2 == 0) return 0;
    uint64_t e1 = seg_end(s1, z1), e2 = seg_end(s2, z2);
    return s1 < e2 && e1 > s2;
}

static int any_overlap(const or_seg *a, int na, const or_seg *b, int nb)
{
    for (int i = 0; i < na; i++)
        for (int j = 0; j < nb; j++)
            if (or_overlap(a[i].start, a[i].size, b[j].start, b[j].size)) return 1;
    return 0;
}

int or_conflict_literal(const or_access *older, const or_access *newer)
{
    /* Algorithm 1 as printed: the incoming kernel's write segments against
     * the read and write segments of a kernel already in the window. */
    return any_overlap(newer->w, newer->n_w, older->r, older->n_r) ||
           any_overlap(newer->w, newer->n_w, older->w, older->n_w);
}

int or_conflict(const or_access *older, const or_access *newer)
{
    /* Reading adopted here: the printed test also has to run the other way
     * (incoming reads against window writes), otherwise a read-after-write
     * pair is not seen as dependent. */
    return or_conflict_literal(older, newer) ||
           any_overlap(newer->r, newer->n_r, older->w, older->n_w);
}

void or_dag(int32_t n, const or_access *acc, int32_t literal, uint8_t *adj)
{
    memset(adj, 0, (size_t)n * (size_t)n);
    for (int32_t j = 0; j < n; j++)
        for (int32_t i = 0; i < j; i++)
            adj[(size_t)i * n + j] = (uint8_t)(literal ? or_conflict_literal(&acc[i], &acc[j])
                                                        : or_conflict(&acc[i], &acc[j]));
}

/* ------------------------------------------------------------------------ */
/* Trace checker                                                              */
/* ------------------------------------------------------------------------ */

#define FAIL(code, ...) do { if (msg && msglen > 0) snprintf(msg, (size_t)msglen, __VA_ARGS__); \
                             free(adj); return (code); } while (0)

int32_t or_check_trace(int32_t n, const or_access *acc, int32_t W, const or_trace_rec *tr,
                       int32_t check_times, int32_t early, char *msg, int32_t msglen)
{
    if (early) check_times = 1;
    if (msg && msglen > 0) msg[0] = 0;
    uint8_t *adj = NULL;
    if (W < 1 || W > 64) FAIL(1, "window size %d outside [1,64]", W);
    if (n <= 0) { return 0; }
    adj = (uint8_t *)malloc((size_t)n * (size_t)n);
    if (!adj) FAIL(2, "out of memory");
    or_dag(n, acc, 0, adj);

    for (int32_t j = 0; j < n; j++) {
        const or_trace_rec *t = &tr[j];
        if (t->seq != j) FAIL(3, "record %d carries seq %lld", j, (long long)t->seq);
        if (t->slot < 0 || t->slot >= W) FAIL(4, "kernel %d in slot %lld outside window %d", j, (long long)t->slot, W);
        if (t->ev_retire < 0) FAIL(5, "kernel %d never retired", j);
        if (!(t->ev_insert < t->ev_dispatch && t->ev_dispatch < t->ev_retire))
            FAIL(6, "kernel %d events out of order: insert %lld dispatch %lld retire %lld", j,
                 (long long)t->ev_insert, (long long)t->ev_dispatch, (long long)t->ev_retire);
        if (j > 0 && !(tr[j - 1].ev_insert < t->ev_insert))
            FAIL(7, "kernel %d admitted before kernel %d (program order broken)", j, j - 1);
        if (t->up_mask & ~t->valid_mask)
            FAIL(8, "kernel %d upstream mask %llx not inside valid mask %llx", j,
                 (unsigned long long)t->up_mask, (unsigned long long)t->valid_mask);
    }

    for (int32_t j = 0; j < n; j++) {
        const or_trace_rec *t = &tr[j];
        uint64_t valid = 0, up = 0;
        int count = 0;
        for (int32_t i = 0; i < j; i++) {
            int in_window = tr[i].ev_insert < t->ev_insert && t->ev_insert < tr[i].ev_retire;
            int dep = adj[(size_t)i * n + j];
            if (in_window) {
                uint64_t bit = 1ull << tr[i].slot;
                if (valid & bit) FAIL(10, "slot %lld held by two kernels at insert of %d", (long long)tr[i].slot, j);
                if (tr[i].slot == t->slot) FAIL(11, "kernel %d inserted into occupied slot %lld", j, (long long)t->slot);
                valid |= bit;
                count++;
                if (dep) up |= bit;
            } else if (dep && !(tr[i].ev_retire < t->ev_insert)) {
                FAIL(12, "kernel %d depends on %d, which was neither in the window nor retired", j, i);
            }
            if (dep && !early && !(tr[i].ev_retire < t->ev_dispatch))
                FAIL(13, "kernel %d dispatched before its upstream kernel %d retired", j, i);
            if (dep && early && !(tr[i].ev_dispatch < t->ev_dispatch))
                FAIL(17, "kernel %d handed out before its upstream kernel %d", j, i);
        }
        if (count > W - 1) FAIL(14, "window held %d kernels besides %d (W=%d)", count, j, W);
        if (valid != t->valid_mask)
            FAIL(15, "kernel %d: recorded valid mask %llx, window was %llx", j,
                 (unsigned long long)t->valid_mask, (unsigned long long)valid);
        if (up != t->up_mask)
            FAIL(16, "kernel %d: recorded upstream mask %llx, dependency check gives %llx", j,
                 (unsigned long long)t->up_mask, (unsigned long long)up);
    }

    if (check_times) {
        for (int32_t j = 0; j < n; j++) {
            if (tr[j].t_start < 0 || tr[j].t_end < tr[j].t_start)
                FAIL(20, "kernel %d has execution interval [%lld,%lld]", j,
                     (long long)tr[j].t_start, (long long)tr[j].t_end);
            for (int32_t i = 0; i < j; i++)
                if (adj[(size_t)i * n + j] && tr[i].t_end > tr[j].t_start)
                    FAIL(21, "conflicting kernels %d and %d overlap in time ([%lld,%lld] vs [%lld,%lld])", i, j,
                         (long long)tr[i].t_start, (long long)tr[i].t_end,
                         (long long)tr[j].t_start, (long long)tr[j].t_end);
        }
    }
    free(adj);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tiny random stream: scale, axpy, sum_reduce                               */
/* ------------------------------------------------------------------------ */

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

void or_tiny_access(const int64_t *offs, const int64_t *lens, uint64_t base,
                    const or_tiny_kernel *k, or_access *acc)
{
    memset(acc, 0, sizeof(*acc));
    if (k->op == OR_OP_SCALE || k->op == OR_OP_AXPY) {
        int64_t n = lens[k->out];
        for (int i = 0; i < k->nin; i++) n = min64(n, lens[k->in[i]]);
        for (int i = 0; i < k->nin; i++) {
            acc->r[acc->n_r].start = base + 4ull * (uint64_t)offs[k->in[i]];
            acc->r[acc->n_r].size = 4ull * (uint64_t)n;
            acc->n_r++;
        }
        acc->w[0].start = base + 4ull * (uint64_t)offs[k->out];
        acc->w[0].size = 4ull * (uint64_t)n;
        acc->n_w = 1;
    } else {
        for (int i = 0; i < k->nin; i++) {
            acc->r[acc->n_r].start = base + 4ull * (uint64_t)offs[k->in[i]];
            acc->r[acc->n_r].size = 4ull * (uint64_t)lens[k->in[i]];
            acc->n_r++;
        }
        acc->w[0].start = base + 4ull * (uint64_t)(offs[k->out] + k->j);
        acc->w[0].size = 4;
        acc->n_w = 1;
    }
}

/* Pairwise sum: pad with zeros to the next power of two P, then for
 * s = P/2, P/4, ..., 1 add element i+s into element i. */
float or_tree_sum(const float *v, int64_t n)
{
    int64_t P = 1;
    while (P < n) P <<= 1;
    float *t = (float *)calloc((size_t)P, sizeof(float));
    memcpy(t, v, (size_t)n * sizeof(float));
    for (int64_t s = P / 2; s >= 1; s /= 2)
        for (int64_t i = 0; i < s; i++) t[i] = t[i] + t[i + s];
    float r = t[0];
    free(t);
    return r;
}

static void tiny_one(float *arena, const int64_t *offs, const int64_t *lens, const or_tiny_kernel *k)
{
    float *out = arena + offs[k->out];
    if (k->op == OR_OP_SCALE) {
        const float *x = arena + offs[k->in[0]];
        int64_t n = min64(lens[k->out], lens[k->in[0]]);
        for (int64_t i = 0; i < n; i++) out[i] = k->a * x[i];
    } else if (k->op == OR_OP_AXPY) {
        const float *x = arena + offs[k->in[0]];
        const float *y = arena + offs[k->in[1]];
        int64_t n = min64(lens[k->out], min64(lens[k->in[0]], lens[k->in[1]]));
        for (int64_t i = 0; i < n; i++) out[i] = fmaf(k->a, x[i], y[i]);
    } else {
        int64_t total = 0;
        for (int i = 0; i < k->nin; i++) total += lens[k->in[i]];
        float *cat = (float *)malloc((size_t)total * sizeof(float));
        int64_t p = 0;
        for (int i = 0; i < k->nin; i++) {
            memcpy(cat + p, arena + offs[k->in[i]], (size_t)lens[k->in[i]] * sizeof(float));
            p += lens[k->in[i]];
        }
        out[k->j] = or_tree_sum(cat, total);
        free(cat);
    }
}

void or_tiny_run(float *arena, const int64_t *offs, const int64_t *lens,
                 int32_t nk, const or_tiny_kernel *ks, const int32_t *order)
{
    for (int32_t q = 0; q < nk; q++) tiny_one(arena, offs, lens, &ks[order ? order[q] : q]);
}

/* ------------------------------------------------------------------------ */
/* Rigid-body RL step                                                         */
/* ------------------------------------------------------------------------ */

/* squared distance with a fixed order: fma(dz,dz, fma(dy,dy, dx*dx)) */
static float dist2(float dx, float dy, float dz)
{
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

static void rl_predict(or_scene *s)
{
    for (int32_t i = 0; i < 4 * s->n; i++) s->P[i] = fmaf(s->dt, s->V[i], s->X[i]);
}

static void rl_broadphase(or_scene *s)
{
    const int32_t n = s->n;
    const float two_r = 2.0f * s->r, thr = two_r * two_r;
    int32_t e = 0;
    for (int32_t i = 0; i < n; i++) {
        s->adj_off[i] = e;
        for (int32_t j = 0; j < n; j++) {
            if (j == i) continue;
            float dx = s->P[4 * i] - s->P[4 * j];
            float dy = s->P[4 * i + 1] - s->P[4 * j + 1];
            float dz = s->P[4 * i + 2] - s->P[4 * j + 2];
            if (dist2(dx, dy, dz) < thr) s->adj[e++] = j;
        }
        s->deg[i] = e - s->adj_off[i];
    }
    s->adj_off[n] = e;
}

static void rl_islands(or_scene *s)
{
    const int32_t n = s->n;
    /* connected components by breadth-first search, visiting roots in index
     * order so that every component is labelled with its smallest body */
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; i++) s->label[i] = -1;
    int32_t n_isl = 0;
    for (int32_t root = 0; root < n; root++) {
        if (s->label[root] >= 0) continue;
        n_isl++;
        int32_t head = 0, tail = 0;
        queue[tail++] = root;
        s->label[root] = root;
        while (head < tail) {
            int32_t b = queue[head++];
            for (int32_t k = s->adj_off[b]; k < s->adj_off[b + 1]; k++) {
                int32_t c = s->adj[k];
                if (s->label[c] < 0) { s->label[c] = root; queue[tail++] = c; }
            }
        }
    }
    free(queue);
    /* islands ordered by their smallest body; bodies inside in index order */
    int32_t pos = 0, k = 0, multi = 0;
    for (int32_t root = 0; root < n; root++) {
        if (s->label[root] != root) continue;
        s->isl_off[k++] = pos;
        for (int32_t b = root; b < n; b++)
            if (s->label[b] == root) { s->perm[pos] = b; s->inv_perm[b] = pos; pos++; }
    }
    s->isl_off[k] = pos;
    /* adjacency in permuted positions */
    int32_t e = 0;
    for (int32_t p = 0; p < n; p++) {
        int32_t b = s->perm[p];
        s->padj_off[p] = e;
        for (int32_t q = s->adj_off[b]; q < s->adj_off[b + 1]; q++) s->padj[e++] = s->inv_perm[s->adj[q]];
    }
    s->padj_off[n] = e;
    for (int32_t i = 0; i < n_isl; i++) {
        int32_t b0 = s->isl_off[i], b1 = s->isl_off[i + 1];
        if (b1 - b0 < 2) continue;
        s->plan[4 * multi + 0] = b0;
        s->plan[4 * multi + 1] = b1;
        s->plan[4 * multi + 2] = s->padj_off[b0];
        s->plan[4 * multi + 3] = s->padj_off[b1];
        multi++;
    }
    s->meta[0] = n_isl;
    s->meta[1] = multi;
    s->meta[2] = e;
}

static void rl_permute(or_scene *s)
{
    for (int32_t p = 0; p < s->n; p++)
        for (int c = 0; c < 4; c++) s->Q0[4 * p + c] = s->P[4 * s->perm[p] + c];
}

static void rl_jacobi(or_scene *s, int32_t island, int32_t iter)
{
    const float *src = (iter % 2 == 0) ? s->Q0 : s->Q1;
    float *dst = (iter % 2 == 0) ? s->Q1 : s->Q0;
    const float two_r = 2.0f * s->r;
    int32_t b0 = s->plan[4 * island], b1 = s->plan[4 * island + 1];
    for (int32_t p = b0; p < b1; p++) {
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
        int32_t e0 = s->padj_off[p], e1 = s->padj_off[p + 1];
        for (int32_t e = e0; e < e1; e++) {
            int32_t q = s->padj[e];
            float dx = src[4 * p] - src[4 * q];
            float dy = src[4 * p + 1] - src[4 * q + 1];
            float dz = src[4 * p + 2] - src[4 * q + 2];
            float d = sqrtf(dist2(dx, dy, dz));
            float pen = two_r - d;
            if (pen > 0.0f) {
                float h = 0.5f * pen, nx, ny, nz;
                if (d > 0.0f) { nx = dx / d; ny = dy / d; nz = dz / d; }
                else { nx = (p < q) ? 1.0f : -1.0f; ny = 0.0f; nz = 0.0f; }
                ax = fmaf(h, nx, ax);
                ay = fmaf(h, ny, ay);
                az = fmaf(h, nz, az);
            }
        }
        float deg = (float)(e1 - e0);
        dst[4 * p] = src[4 * p] + ax / deg;
        dst[4 * p + 1] = src[4 * p + 1] + ay / deg;
        dst[4 * p + 2] = src[4 * p + 2] + az / deg;
        dst[4 * p + 3] = src[4 * p + 3];
    }
}

static void rl_integrate(or_scene *s)
{
    const float lo = s->r, hi = 1.0f - s->r;
    for (int32_t i = 0; i < s->n; i++) {
        int32_t p = s->inv_perm[i];
        for (int c = 0; c < 3; c++) {
            float x = s->Q0[4 * p + c];
            float v = s->V[4 * i + c] + (x - s->P[4 * i + c]) / s->dt;
            if (x < lo) { x = lo; v = fabsf(v); }
            else if (x > hi) { x = hi; v = -fabsf(v); }
            s->X[4 * i + c] = x;
            s->V[4 * i + c] = v;
        }
        s->X[4 * i + 3] = s->Q0[4 * p + 3];
    }
}

void or_rl_run_kernel(or_scene *s, const or_rl_kernel *k)
{
    switch (k->op) {
    case OR_RL_PREDICT: rl_predict(s); break;
    case OR_RL_BROADPHASE: rl_broadphase(s); break;
    case OR_RL_ISLANDS: rl_islands(s); break;
    case OR_RL_PERMUTE: rl_permute(s); break;
    case OR_RL_JACOBI: rl_jacobi(s, k->island, k->iter); break;
    case OR_RL_INTEGRATE: rl_integrate(s); break;
    default: break;
    }
}

/* Accesses in a private address space: buffer b occupies [b << 40, ...). */
enum { RG_X = 1, RG_V, RG_P, RG_Q0, RG_Q1, RG_DEG, RG_ADJOFF, RG_ADJ, RG_LABEL, RG_PERM,
       RG_INVPERM, RG_ISLOFF, RG_PADJOFF, RG_PADJ, RG_META, RG_PLAN };

static void add_seg(or_seg *list, int32_t *cnt, int region, uint64_t off, uint64_t size)
{
    list[*cnt].start = ((uint64_t)region << 40) + off;
    list[*cnt].size = size;
    (*cnt)++;
}

void or_rl_access(const or_scene *s, const or_rl_kernel *k, or_access *a)
{
    const uint64_t n = (uint64_t)s->n, vec = 16 * n, ints = 4 * n, edges = 4 * n * (n - 1);
    memset(a, 0, sizeof(*a));
    switch (k->op) {
    case OR_RL_PREDICT:
        add_seg(a->r, &a->n_r, RG_X, 0, vec);
        add_seg(a->r, &a->n_r, RG_V, 0, vec);
        add_seg(a->w, &a->n_w, RG_P, 0, vec);
        break;
    case OR_RL_BROADPHASE:
        add_seg(a->r, &a->n_r, RG_P, 0, vec);
        add_seg(a->w, &a->n_w, RG_DEG, 0, ints);
        add_seg(a->w, &a->n_w, RG_ADJOFF, 0, ints + 4);
        add_seg(a->w, &a->n_w, RG_ADJ, 0, edges);
        break;
    case OR_RL_ISLANDS:
        add_seg(a->r, &a->n_r, RG_DEG, 0, ints);
        add_seg(a->r, &a->n_r, RG_ADJOFF, 0, ints + 4);
        add_seg(a->r, &a->n_r, RG_ADJ, 0, edges);
        add_seg(a->w, &a->n_w, RG_LABEL, 0, ints);
        add_seg(a->w, &a->n_w, RG_PERM, 0, ints);
        add_seg(a->w, &a->n_w, RG_INVPERM, 0, ints);
        add_seg(a->w, &a->n_w, RG_ISLOFF, 0, ints + 4);
        add_seg(a->w, &a->n_w, RG_PADJOFF, 0, ints + 4);
        add_seg(a->w, &a->n_w, RG_PADJ, 0, edges);
        add_seg(a->w, &a->n_w, RG_META, 0, 12);
        add_seg(a->w, &a->n_w, RG_PLAN, 0, 16 * (n / 2));
        break;
    case OR_RL_PERMUTE:
        add_seg(a->r, &a->n_r, RG_P, 0, vec);
        add_seg(a->r, &a->n_r, RG_PERM, 0, ints);
        add_seg(a->w, &a->n_w, RG_Q0, 0, vec);
        break;
    case OR_RL_JACOBI: {
        uint64_t b0 = (uint64_t)s->plan[4 * k->island], b1 = (uint64_t)s->plan[4 * k->island + 1];
        uint64_t e0 = (uint64_t)s->plan[4 * k->island + 2], e1 = (uint64_t)s->plan[4 * k->island + 3];
        int src = (k->iter % 2 == 0) ? RG_Q0 : RG_Q1, dst = (k->iter % 2 == 0) ? RG_Q1 : RG_Q0;
        add_seg(a->r, &a->n_r, src, 16 * b0, 16 * (b1 - b0));
        add_seg(a->r, &a->n_r, RG_PADJOFF, 4 * b0, 4 * (b1 - b0 + 1));
        add_seg(a->r, &a->n_r, RG_PADJ, 4 * e0, 4 * (e1 - e0));
        add_seg(a->w, &a->n_w, dst, 16 * b0, 16 * (b1 - b0));
        break;
    }
    case OR_RL_INTEGRATE:
        add_seg(a->r, &a->n_r, RG_P, 0, vec);
        add_seg(a->r, &a->n_r, RG_V, 0, vec);
        add_seg(a->r, &a->n_r, RG_Q0, 0, vec);
        add_seg(a->r, &a->n_r, RG_INVPERM, 0, ints);
        add_seg(a->w, &a->n_w, RG_X, 0, vec);
        add_seg(a->w, &a->n_w, RG_V, 0, vec);
        break;
    default: break;
    }
}

int32_t or_rl_step_kernels(const or_scene *s, or_rl_kernel *out, int32_t cap)
{
    int32_t c = 0;
#define PUSH(o, isl, it) do { if (c < cap) { out[c].op = (o); out[c].island = (isl); out[c].iter = (it); } c++; } while (0)
    PUSH(OR_RL_PREDICT, 0, 0);
    PUSH(OR_RL_BROADPHASE, 0, 0);
    PUSH(OR_RL_ISLANDS, 0, 0);
    PUSH(OR_RL_PERMUTE, 0, 0);
    for (int32_t t = 0; t < s->iters; t++)
        for (int32_t k = 0; k < s->meta[1]; k++) PUSH(OR_RL_JACOBI, k, t);
    PUSH(OR_RL_INTEGRATE, 0, 0);
#undef PUSH
    return c;
}

void or_rl_step(or_scene *s)
{
    or_rl_kernel k = {0, 0, 0};
    k.op = OR_RL_PREDICT; or_rl_run_kernel(s, &k);
    k.op = OR_RL_BROADPHASE; or_rl_run_kernel(s, &k);
    k.op = OR_RL_ISLANDS; or_rl_run_kernel(s, &k);
    k.op = OR_RL_PERMUTE; or_rl_run_kernel(s, &k);
    for (int32_t t = 0; t < s->iters; t++)
        for (int32_t i = 0; i < s->meta[1]; i++) {
            k.op = OR_RL_JACOBI; k.island = i; k.iter = t;
            or_rl_run_kernel(s, &k);
        }
    k.op = OR_RL_INTEGRATE; or_rl_run_kernel(s, &k);
}

/* ------------------------------------------------------------------------- */
/* Dynamic DNN (Section II-C), batch 1, NHWC                                 */
/* ------------------------------------------------------------------------- */

int32_t or_conv_hout(int32_t hin, int32_t k, int32_t s)
{
    const int32_t p = (k - 1) / 2;
    return (hin + 2 * p - k) / s + 1;
}

void or_conv_f32(const float *in, const float *w, const float *b, float *out,
                 int32_t hin, int32_t cin, int32_t cout, int32_t k, int32_t s)
{
    const int32_t p = (k - 1) / 2, hout = or_conv_hout(hin, k, s);
    for (int32_t y = 0; y < hout; y++)
        for (int32_t x = 0; x < hout; x++)
            for (int32_t co = 0; co < cout; co++) {
                float acc = 0.0f;
                for (int32_t ky = 0; ky < k; ky++)
                    for (int32_t kx = 0; kx < k; kx++) {
                        const int32_t iy = y * s + ky - p, ix = x * s + kx - p;
                        for (int32_t ci = 0; ci < cin; ci++) {
                            const float a = (iy >= 0 && iy < hin && ix >= 0 && ix < hin)
                                                ? in[((int64_t)iy * hin + ix) * cin + ci] : 0.0f;
                            acc = fmaf(a, w[(((int64_t)ky * k + kx) * cin + ci) * cout + co], acc);
                        }
                    }
                out[((int64_t)y * hout + x) * cout + co] = acc + b[co];
            }
}

void or_conv_f64(const float *in, const float *w, const float *b, double *out, double *mag,
                 int32_t hin, int32_t cin, int32_t cout, int32_t k, int32_t s)
{
    const int32_t p = (k - 1) / 2, hout = or_conv_hout(hin, k, s);
    for (int32_t y = 0; y < hout; y++)
        for (int32_t x = 0; x < hout; x++)
            for (int32_t co = 0; co < cout; co++) {
                double acc = (double)b[co], m = fabs((double)b[co]);
                for (int32_t ky = 0; ky < k; ky++)
                    for (int32_t kx = 0; kx < k; kx++) {
                        const int32_t iy = y * s + ky - p, ix = x * s + kx - p;
                        if (iy < 0 || iy >= hin || ix < 0 || ix >= hin) continue;
                        for (int32_t ci = 0; ci < cin; ci++) {
                            const double t = (double)in[((int64_t)iy * hin + ix) * cin + ci] *
                                             (double)w[(((int64_t)ky * k + kx) * cin + ci) * cout + co];
                            acc += t;
                            m += fabs(t);
                        }
                    }
                out[((int64_t)y * hout + x) * cout + co] = acc;
                mag[((int64_t)y * hout + x) * cout + co] = m;
            }
}

float or_relu(float x) { return x > 0.0f ? x : 0.0f; }

void or_join(float *out, const float *a, const float *b, int64_t n)
{
    for (int64_t i = 0; i < n; i++) out[i] = or_relu(b ? a[i] + b[i] : a[i]);
}

void or_avgpool(float *out, const float *in, int32_t hw, int32_t c)
{
    for (int32_t ch = 0; ch < c; ch++) {
        float acc = 0.0f;
        for (int32_t q = 0; q < hw; q++) acc += in[(int64_t)q * c + ch];
        out[ch] = acc / (float)hw;
    }
}

void or_fc(float *out, const float *in, const float *w, const float *b, int32_t cin, int32_t cout)
{
    for (int32_t j = 0; j < cout; j++) {
        float acc = b[j];
        for (int32_t i = 0; i < cin; i++) acc = fmaf(in[i], w[(int64_t)i * cout + j], acc);
        out[j] = acc;
    }
}
