// The C ABI (include/acs.h): argument checks, submission normalisation
// (step a1) and dispatch to the chosen path.
#include <string.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "internal.hpp"
#include "launch.hpp"
#include "rl_layout.hpp"


namespace acs {

namespace {
thread_local int t_last_error = ACS_OK;
thread_local std::string t_last_msg;

struct Range {
    uint64_t s, e;
};

// A small list of ranges on the stack (submissions rarely carry more than a
// handful); larger lists spill to the heap.
struct RangeList {
    Range fixed[32];
    std::vector<Range> heap;
    Range *v = fixed;
    size_t n = 0, cap = 32;
    void push(Range r)
    {
        if (n == cap) {
            // copy into a new vector first: v may point into heap itself
            std::vector<Range> grown(cap * 2);
            std::copy(v, v + n, grown.begin());
            heap.swap(grown);
            cap *= 2;
            v = heap.data();
        }
        v[n++] = r;
    }
};

// Sorts and merges overlapping or touching ranges (exact: the union is
// unchanged), then, while more than `budget` remain, merges the neighbours
// with the smallest gap (conservative: the union only grows).
bool shrink(RangeList &L, size_t budget)
{
    Range *v = L.v;
    for (size_t i = 1; i < L.n; i++) {   // insertion sort: lists are short
        Range x = v[i];
        size_t j = i;
        while (j > 0 && (v[j - 1].s > x.s || (v[j - 1].s == x.s && v[j - 1].e > x.e))) {
            v[j] = v[j - 1];
            j--;
        }
        v[j] = x;
    }
    size_t m = 0;
    for (size_t i = 0; i < L.n; i++) {
        if (m > 0 && v[i].s <= v[m - 1].e) {
            if (v[i].e > v[m - 1].e) v[m - 1].e = v[i].e;
        } else {
            v[m++] = v[i];
        }
    }
    bool lossy = false;
    while (m > budget && m > 1) {
        size_t best = 0;
        uint64_t gap = UINT64_MAX;
        for (size_t i = 0; i + 1 < m; i++) {
            const uint64_t g = v[i + 1].s - v[i].e;
            if (g < gap) {
                gap = g;
                best = i;
            }
        }
        if (v[best + 1].e > v[best].e) v[best].e = v[best + 1].e;
        for (size_t i = best + 1; i + 1 < m; i++) v[i] = v[i + 1];
        m--;
        lossy = true;
    }
    L.n = m;
    return lossy;
}

size_t args_size_of(int32_t kid)
{
    switch (kid) {
    case ACS_K_NOP: return sizeof(acs_args_nop);
    case ACS_K_SCALE: return sizeof(acs_args_scale);
    case ACS_K_AXPY: return sizeof(acs_args_axpy);
    case ACS_K_SUM: return sizeof(acs_args_sum);
    case ACS_K_RL_PREDICT:
    case ACS_K_RL_BROADPHASE:
    case ACS_K_RL_ISLANDS:
    case ACS_K_RL_PERMUTE:
    case ACS_K_RL_JACOBI:
    case ACS_K_RL_INTEGRATE: return sizeof(acs_args_rl);
    case ACS_K_CONV: return sizeof(acs_args_conv);
    case ACS_K_JOIN: return sizeof(acs_args_join);
    case ACS_K_AVGPOOL: return sizeof(acs_args_avgpool);
    case ACS_K_FC: return sizeof(acs_args_fc);
    case ACS_K_COPY: return sizeof(acs_args_copy);
    case ACS_K_SIGNAL: return sizeof(acs_args_signal);
    default: return 0;
    }
}

uint32_t div_up(uint32_t a, uint32_t b) { return (a + b - 1) / b; }

// Checks the bounds the bodies rely on and picks the piece count.
bool check_args(int32_t kid, const uint8_t *args, int32_t g, uint32_t &np, std::string *why)
{
    np = 1;
    const uint32_t gg = (uint32_t)std::max(1, std::min(g, 256));
    switch (kid) {
    case ACS_K_SCALE: {
        acs_args_scale a;
        memcpy(&a, args, sizeof(a));
        np = std::max(1u, std::min(gg, div_up(a.n, 256)));
        return true;
    }
    case ACS_K_AXPY: {
        acs_args_axpy a;
        memcpy(&a, args, sizeof(a));
        np = std::max(1u, std::min(gg, div_up(a.n, 256)));
        return true;
    }
    case ACS_K_SUM: {
        acs_args_sum a;
        memcpy(&a, args, sizeof(a));
        uint64_t tot = 0;
        if (a.nin < 1 || a.nin > 3) {
            if (why) *why = "sum: nin must be 1..3";
            return false;
        }
        for (uint32_t k = 0; k < a.nin; k++) tot += a.len[k];
        if (tot == 0 || tot > 256u * 64u) {
            if (why) *why = "sum: total length must be in [1, 16384]";
            return false;
        }
        return true;
    }
    case ACS_K_RL_PREDICT:
    case ACS_K_RL_BROADPHASE:
    case ACS_K_RL_ISLANDS:
    case ACS_K_RL_PERMUTE:
    case ACS_K_RL_JACOBI:
    case ACS_K_RL_INTEGRATE: {
        acs_args_rl a;
        memcpy(&a, args, sizeof(a));
        if (a.n < 2 || a.n > kRLMaxBodies) {
            if (why) *why = "rl: n must be in [2, 1024]";
            return false;
        }
        if (kid == ACS_K_RL_JACOBI && (a.b0 < 0 || a.b1 > a.n || a.b0 >= a.b1 || a.iter < 0)) {
            if (why) *why = "rl jacobi: bad island range";
            return false;
        }
        if (kid == ACS_K_RL_ISLANDS && a.plan == 0) {
            if (why) *why = "rl islands: plan buffer missing";
            return false;
        }
        if (kid == ACS_K_RL_PREDICT || kid == ACS_K_RL_PERMUTE || kid == ACS_K_RL_INTEGRATE)
            np = std::max(1u, std::min(gg, div_up((uint32_t)a.n, 256)));
        return true;
    }
    case ACS_K_CONV: {
        acs_args_conv a;
        memcpy(&a, args, sizeof(a));
        if ((a.k != 1 && a.k != 3) || (a.stride != 1 && a.stride != 2) || a.hin < 1 || a.hin > 4096 ||
            a.cin < 32 || a.cin % 32 != 0 || a.cout < 32 || a.cout % 32 != 0 || a.cin > 4096 || a.cout > 4096 ||
            !a.in || !a.w || !a.bias || !a.out) {
            if (why) *why = "conv: k in {1,3}, stride in {1,2}, cin and cout multiples of 32, non-null buffers";
            return false;
        }
        const int64_t pad = (a.k - 1) / 2, hout = (a.hin + 2 * pad - a.k) / a.stride + 1, m = hout * hout;
        if (hout < 1 || m % 16 != 0) {
            if (why) *why = "conv: output pixels must be a multiple of 16";
            return false;
        }
        // one piece per 16 x 32 output tile, at most 256 pieces (tiles are dealt round-robin)
        np = (uint32_t)std::min<int64_t>((m / 16) * (a.cout / 32), 256);
        return true;
    }
    case ACS_K_JOIN: {
        acs_args_join a;
        memcpy(&a, args, sizeof(a));
        if (!a.out || !a.a) {
            if (why) *why = "join: null buffer";
            return false;
        }
        // one piece per 2048 elements (an activation tensor is not a small body)
        np = std::max(1u, std::min(256u, div_up(a.n, 2048)));
        return true;
    }
    case ACS_K_AVGPOOL: {
        acs_args_avgpool a;
        memcpy(&a, args, sizeof(a));
        if (a.hw < 1 || a.c < 1 || a.c > 4096 || !a.in || !a.out) {
            if (why) *why = "avgpool: bad shape";
            return false;
        }
        return true;
    }
    case ACS_K_FC: {
        acs_args_fc a;
        memcpy(&a, args, sizeof(a));
        if (a.cin < 1 || a.cout < 1 || a.cout > 4096 || !a.in || !a.w || !a.bias || !a.out) {
            if (why) *why = "fc: bad shape";
            return false;
        }
        return true;
    }
    case ACS_K_COPY: {
        acs_args_copy a;
        memcpy(&a, args, sizeof(a));
        const uint64_t d = (uint64_t)(uintptr_t)a.dst, s = (uint64_t)(uintptr_t)a.src;
        if (!a.dst || !a.src || (d | s | a.bytes) % 16 != 0 || a.bytes > (1ull << 40) || (d < s + a.bytes && s < d + a.bytes)) {
            if (why) *why = "copy: null, unaligned or overlapping buffers";
            return false;
        }
        np = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(gg, (a.bytes + 4095) / 4096));
        return true;
    }
    case ACS_K_SIGNAL: {
        acs_args_signal a;
        memcpy(&a, args, sizeof(a));
        if (!a.addr || (uint64_t)(uintptr_t)a.addr % 8 != 0) {
            if (why) *why = "signal: null or unaligned word";
            return false;
        }
        return true;
    }
    default: return true;
    }
}
}  // namespace

void set_error(int code, const std::string &msg)
{
    t_last_error = code;
    t_last_msg = msg;
}

int make_desc(int32_t kid, const acs_seg *r, int32_t nr, const acs_seg *w, int32_t nw, const void *args,
              size_t args_size, int32_t wg_per_task, Desc &out, bool *coalesced, std::string *why)
{
    const size_t want = args_size_of(kid);
    if (want == 0) {
        *why = "unknown kernel id";
        return ACS_EINVAL;
    }
    if (args_size != want || args == nullptr) {
        *why = "args_size does not match the task's argument struct";
        return ACS_EINVAL;
    }
    if (nr < 0 || nw < 0 || (nr > 0 && !r) || (nw > 0 && !w)) {
        *why = "bad segment list";
        return ACS_EINVAL;
    }
    RangeList rr, ww;
    auto take = [&](const acs_seg *lst, int32_t n, RangeList &dst) -> bool {
        for (int32_t i = 0; i < n; i++) {
            const uint64_t st = lst[i].start, z = lst[i].size;
            if (z == 0) continue;
            uint64_t e;
            if (z > UINT64_MAX - st) {
                if (st == ACS_SEG_ALL_START && z == ACS_SEG_ALL_SIZE)
                    e = UINT64_MAX;
                else
                    return false;
            } else {
                e = st + z;
            }
            dst.push({st, e});
        }
        return true;
    };
    if (!take(r, nr, rr) || !take(w, nw, ww)) {
        *why = "segment wraps past the end of the address space";
        return ACS_EINVAL;
    }
    bool lossy = shrink(rr, ACS_K_MAX);
    lossy |= shrink(ww, ACS_K_MAX);
    while (rr.n + ww.n > ACS_K_MAX) {
        // give the writes at least half of the budget, the reads the rest
        const size_t wbud = std::min(ww.n, (size_t)std::max<int>(ACS_K_MAX / 2, ACS_K_MAX - (int)rr.n));
        lossy |= shrink(ww, std::max<size_t>(1, wbud));
        lossy |= shrink(rr, ACS_K_MAX - ww.n);
    }
    out.kid = kid;
    memcpy(out.args, args, args_size);
    if (args_size < ACS_ARGS_MAX) memset(out.args + args_size, 0, ACS_ARGS_MAX - args_size);
    out.args_size = (uint32_t)args_size;
    // writes first: a read only has to be tested against the first
    // positions of the other kernels, up to the most writes any kernel has
    out.wbits = 0;
    uint32_t k = 0;
    for (size_t i = 0; i < ww.n; i++, k++) {
        out.s[k] = ww.v[i].s;
        out.e[k] = ww.v[i].e;
        out.wbits |= 1u << k;
    }
    for (size_t i = 0; i < rr.n; i++, k++) {
        out.s[k] = rr.v[i].s;
        out.e[k] = rr.v[i].e;
    }
    out.nseg = k;
    for (; k < ACS_K_MAX; k++) out.s[k] = out.e[k] = 0;
    uint32_t np = 1;
    if (!check_args(kid, out.args, wg_per_task, np, why)) return ACS_EINVAL;
    out.npieces = np;
    if (coalesced) *coalesced = lossy;
    return ACS_OK;
}

}  // namespace acs

using namespace acs;

namespace {
int fail(int code, const std::string &msg)
{
    set_error(code, msg);
    return code;
}

int ensure_started(acs_window *w)
{
    if (w->started) return ACS_OK;
    if (!w->configured) acs_config_default(&w->cfg);
    switch (w->cfg.path) {
    case ACS_PATH_INORDER: w->path = make_inorder_path(w->cfg); break;
    // groups share one host window on the plain and manual paths (valid
    // because kernels of different groups touch disjoint memory)
    case ACS_PATH_PLAIN: w->path = make_plain_path(std::min(ACS_W_MAX, w->W * w->cfg.n_groups), w->cfg); break;
    case ACS_PATH_DEVICE: w->path = make_device_path(w->W, w->cfg); break;
    case ACS_PATH_MANUAL: w->path = make_manual_path(std::min(ACS_W_MAX, w->W * w->cfg.n_groups), w->cfg); break;
    case ACS_PATH_EVENTS: w->path = make_events_path(w->cfg); break;
    default: return fail(ACS_EINVAL, "unknown path");
    }
    const int rc = w->path->start();
    if (rc != ACS_OK) {
        w->path.reset();
        return rc;
    }
    w->started = true;
    return ACS_OK;
}

int validate_config(const acs_window *w, const acs_config *cfg)
{
    if (cfg->path < ACS_PATH_INORDER || cfg->path > ACS_PATH_EVENTS) return fail(ACS_EINVAL, "unknown path");
    if (cfg->n_streams < 1 || cfg->n_streams > 64) return fail(ACS_EINVAL, "n_streams must be in [1, 64]");
    if (cfg->wg_per_task < 1 || cfg->wg_per_task > 256) return fail(ACS_EINVAL, "wg_per_task must be in [1, 256]");
    if (cfg->n_workers < 0 || cfg->n_workers > 8192) return fail(ACS_EINVAL, "n_workers must be in [0, 8192]");
    if (cfg->queue_depth < 1 || cfg->queue_depth > (1 << 20)) return fail(ACS_EINVAL, "queue_depth must be in [1, 2^20]");
    if (cfg->trace && (cfg->trace_capacity < 1 || cfg->trace_capacity > (1 << 24)))
        return fail(ACS_EINVAL, "trace_capacity must be in [1, 2^24]");
    if (cfg->n_groups < 1 || cfg->n_groups > 8) return fail(ACS_EINVAL, "n_groups must be in [1, 8]");
    if (cfg->path == ACS_PATH_DEVICE) {
        int32_t wp = 1;
        while (wp < w->W) wp <<= 1;
        if (wp * cfg->n_groups > ACS_W_MAX)
            return fail(ACS_EINVAL, "device path: n_groups times W rounded up to a power of two must be at most 64");
    }
    if (cfg->host_check_depth < 0 || cfg->host_check_depth > ACS_HOST_CHECK_MAX)
        return fail(ACS_EINVAL, "host_check_depth must be in [0, " + std::to_string(ACS_HOST_CHECK_MAX) + "]");
    if (cfg->path == ACS_PATH_DEVICE && cfg->host_check_depth > 0 && cfg->n_groups != 1)
        return fail(ACS_EINVAL, "host checks need a single window group");
    if (cfg->window_check != 0 && cfg->window_check != 1) return fail(ACS_EINVAL, "window_check must be 0 or 1");
    return ACS_OK;
}
}  // namespace

extern "C" {

void acs_config_default(acs_config *cfg)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->path = ACS_PATH_DEVICE;
    cfg->n_streams = 4;
    cfg->wg_per_task = 1;
    cfg->n_workers = 0;
    cfg->queue_depth = 4096;
    cfg->nonblocking = 0;
    cfg->trace = 0;
    cfg->trace_capacity = 1 << 16;
    cfg->device = 0;
    cfg->n_groups = 1;
}

acs_window *acs_window_create(int32_t W)
{
    if (W < 1 || W > ACS_W_MAX) {
        set_error(ACS_EINVAL, "window size must be in [1, 64]");
        return nullptr;
    }
    acs_window *w = new (std::nothrow) acs_window();
    if (!w) {
        set_error(ACS_ENOMEM, "out of memory");
        return nullptr;
    }
    w->W = W;
    acs_config_default(&w->cfg);
    return w;
}

int acs_window_configure(acs_window *w, const acs_config *cfg)
{
    if (!w || !cfg) return fail(ACS_EINVAL, "null argument");
    if (w->started) return fail(ACS_ESTATE, "configure must come before the first submit");
    if (int rc = validate_config(w, cfg)) return rc;
    w->cfg = *cfg;
    w->configured = true;
    return ensure_started(w);
}

int acs_window_configure_noalloc(acs_window *w, const acs_config *cfg, void *host_mem, uint64_t host_bytes,
                                 void *stream)
{
    if (!w || !cfg || !host_mem || !stream) return fail(ACS_EINVAL, "null argument");
    if (w->started) return fail(ACS_ESTATE, "configure must come before the first submit");
    if (int rc = validate_config(w, cfg)) return rc;
    if (cfg->path != ACS_PATH_DEVICE) return fail(ACS_EINVAL, "only the device path has a configuration without allocation");
    if (reinterpret_cast<uintptr_t>(host_mem) % 64 != 0) return fail(ACS_EINVAL, "host block must be 64-byte aligned");
    int rc = ACS_OK;
    std::unique_ptr<Path> p = make_device_path_static(w->W, *cfg, host_mem, host_bytes, stream, &rc);
    if (!p) return rc;
    if ((rc = p->start()) != ACS_OK) return rc;   // destroying p releases the device's state
    w->cfg = *cfg;
    w->configured = true;
    w->path = std::move(p);
    w->started = true;
    return ACS_OK;
}

int acs_submit(acs_window *w, int32_t kernel_id, const acs_seg *read_segs, int32_t n_read, const acs_seg *write_segs,
               int32_t n_write, const void *args, size_t args_size, uint64_t *seq_out)
{
    return acs_submit_group(w, 0, kernel_id, read_segs, n_read, write_segs, n_write, args, args_size, seq_out);
}

int acs_submit_group(acs_window *w, int32_t group, int32_t kernel_id, const acs_seg *read_segs, int32_t n_read,
                     const acs_seg *write_segs, int32_t n_write, const void *args, size_t args_size, uint64_t *seq_out)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (w->stopped) return fail(ACS_ESTATE, "window was stopped");
    if (int rc = ensure_started(w)) return rc;
    if (group < 0 || group >= w->cfg.n_groups) return fail(ACS_EINVAL, "group outside [0, n_groups)");
    Desc d;
    bool lossy = false;
    std::string why;
    int rc = make_desc(kernel_id, read_segs, n_read, write_segs, n_write, args, args_size, w->cfg.wg_per_task, d, &lossy,
                       &why);
    if (rc != ACS_OK) return fail(rc, why);
    d.seq = w->next_seq;
    if (w->recording) {
        w->recorded.push_back(d);
        if (lossy) w->coalesced++;
        if (seq_out) *seq_out = d.seq;
        w->next_seq++;
        return ACS_OK;
    }
    rc = w->path->submit_group(d, group);
    if (rc != ACS_OK) return rc;
    if (lossy) w->coalesced++;
    if (seq_out) *seq_out = d.seq;
    w->next_seq++;
    return ACS_OK;
}

int acs_sync(acs_window *w)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (!w->started) return ACS_OK;
    return w->path->sync(0);
}

int acs_sync_timeout(acs_window *w, uint64_t timeout_ns)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (!w->started) return ACS_OK;
    return w->path->sync(timeout_ns == 0 ? 1 : timeout_ns);
}

int acs_sync_group(acs_window *w, int32_t group, uint64_t timeout_ns)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (group < 0 || group >= w->cfg.n_groups) return fail(ACS_EINVAL, "group outside [0, n_groups)");
    if (!w->started) return ACS_OK;
    return w->path->sync_group(group, timeout_ns);
}

int acs_poll(acs_window *w)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (!w->started) return ACS_OK;
    return w->path->poll();
}

int acs_scheduled_list(acs_window *w, acs_entry *out, int32_t cap, int32_t *n_out)
{
    if (!w || (cap > 0 && !out)) return fail(ACS_EINVAL, "bad argument");
    if (!w->started) {
        if (n_out) *n_out = 0;
        return ACS_OK;
    }
    return w->path->scheduled_list(out, cap, n_out);
}

int acs_trace_read(acs_window *w, acs_trace_rec *out, int64_t cap, int64_t *n_out)
{
    if (!w || (cap > 0 && !out)) return fail(ACS_EINVAL, "bad argument");
    if (!w->cfg.trace) return fail(ACS_ESTATE, "tracing is off");
    if (!w->started) {
        if (n_out) *n_out = 0;
        return ACS_OK;
    }
    return w->path->trace_read(out, cap, n_out);
}

int acs_stats_get(acs_window *w, acs_stats *s)
{
    if (!w || !s) return fail(ACS_EINVAL, "bad argument");
    memset(s, 0, sizeof(*s));
    s->submitted = w->next_seq;
    s->coalesced = w->coalesced;
    s->path = w->cfg.path;
    s->W = w->W;
    if (w->started) w->path->stats(*s);
    return ACS_OK;
}

int acs_window_stop(acs_window *w)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (w->stopped) return ACS_OK;
    w->stopped = true;
    if (!w->started) return ACS_OK;
    return w->path->stop();
}

int acs_window_destroy(acs_window *w)
{
    if (!w) return ACS_OK;
    int rc = ACS_OK;
    if (w->started && w->path) {
        if (w->cfg.path != ACS_PATH_MANUAL) rc = w->path->sync(30ull * 1000000000ull);
        const int rc2 = w->path->shutdown();
        if (rc == ACS_OK) rc = rc2;
    }
    delete w;
    return rc;
}

int acs_manual_take_ready(acs_window *w, uint64_t *seqs, int32_t cap, int32_t *n_out)
{
    if (!w || (cap > 0 && !seqs)) return fail(ACS_EINVAL, "bad argument");
    if (int rc = ensure_started(w)) return rc;
    if (w->cfg.path != ACS_PATH_MANUAL) return fail(ACS_ESTATE, "not a manual window");
    return w->path->take_ready(seqs, cap, n_out);
}

int acs_manual_complete(acs_window *w, uint64_t seq, int32_t status)
{
    if (!w) return fail(ACS_EINVAL, "null window");
    if (int rc = ensure_started(w)) return rc;
    if (w->cfg.path != ACS_PATH_MANUAL) return fail(ACS_ESTATE, "not a manual window");
    return w->path->complete(seq, status);
}

void *acs_host_alloc(size_t bytes)
{
    void *p = nullptr;
    const hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) {
        set_error(ACS_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        return nullptr;
    }
    return p;
}

int acs_host_free(void *p)
{
    if (!p) return ACS_OK;
    const hipError_t e = hipHostFree(p);
    return e == hipSuccess ? ACS_OK : fail(ACS_EDEVICE, std::string("hipHostFree: ") + hipGetErrorString(e));
}

int acs_last_error(void) { return t_last_error; }

const char *acs_strerror(int code)
{
    if (code == t_last_error && !t_last_msg.empty()) return t_last_msg.c_str();
    switch (code) {
    case ACS_OK: return "ok";
    case ACS_EINVAL: return "invalid argument";
    case ACS_ENOMEM: return "out of memory";
    case ACS_EAGAIN: return "input FIFO full";
    case ACS_EDEVICE: return "device error";
    case ACS_ETIMEDOUT: return "timed out";
    case ACS_EKERNEL: return "a kernel failed";
    case ACS_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

int acs_device_query(int32_t device, acs_device_info *out)
{
    if (!out) return fail(ACS_EINVAL, "null argument");
    memset(out, 0, sizeof(*out));
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return fail(ACS_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess) out->compute_units = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, device) == hipSuccess) out->wall_clock_khz = v;
    if (hipRuntimeGetVersion(&v) == hipSuccess) out->runtime_version = v;
    int32_t b = 0;
    if (persistent_blocks_per_cu(1, &b) == hipSuccess) out->persistent_wg_per_cu = b;
    if (persistent_lds_bytes(1, &b) == hipSuccess) out->lds_bytes_per_wg = b;
    return ACS_OK;
}

int acs_rl_layout(int32_t n, uint64_t *off)
{
    if (n < 2 || n > kRLMaxBodies || !off) return ACS_EINVAL;
    rl_offsets(n, off);
    return ACS_OK;
}

}  // extern "C"
