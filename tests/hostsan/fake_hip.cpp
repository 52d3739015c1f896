// Host-only stand-in for the HIP runtime calls of libacs's host sources, so
// that those sources can be built with the address and undefined-behaviour
// sanitizers and driven on a machine without a GPU.  Test infrastructure
// only.
//
// Model:
//   - device and pinned memory are host allocations; every pointer handed
//     out is tracked, and freeing an unknown pointer aborts;
//   - a stream is a queue of host closures.  Work runs only when the host
//     queries or synchronises (a query runs a pseudo-random few operations),
//     so completion order and timing differ from submission order the way
//     they do on a device;
//   - events complete when their record operation runs; a wait on an event
//     drives the event's stream until it has;
//   - a graph copies each node's arguments when the node is added (sized by
//     the task's argument struct, as the runtime sizes them from the kernel's
//     signature) and runs its nodes in insertion order, which must be a
//     topological order;
//   - kernels: NOP does nothing, COPY and SIGNAL run on the host, and every
//     other task calls an optional hook (the drivers' tests use it to write
//     the island plan an islands kernel would write).
// Any call on a destroyed stream, event, graph or executable graph aborts
// with a message: on a real device that is undefined behaviour.
#include "hip/hip_runtime_api.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <list>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <vector>

#include "acs_tasks.h"
#include "launch.hpp"

namespace {

[[noreturn]] void die(const char *what)
{
    fprintf(stderr, "fake HIP: %s\n", what);
    fflush(stderr);
    abort();
}

std::recursive_mutex g_mu;   // the library is single-threaded per window; the fake guards itself anyway
uint64_t g_rng = 0x9E3779B97F4A7C15ull;
uint64_t g_clock = 0;
uint64_t rnd()
{
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return g_rng;
}

std::set<void *> g_dev, g_host;

using Op = std::function<void()>;

}  // namespace

struct ihipStream_t {
    std::list<Op> q;   // nodes are freed as operations run
};

struct ihipEvent_t {
    bool pending = false;   // a record operation is queued and has not run
    uint64_t t = 0;         // fake time of the last completed record
    hipStream_t stream = nullptr;
    unsigned flags = 0;
};

struct hipGraphNode {
    int32_t kid = 0;
    std::vector<uint8_t> args;
    uint32_t np = 0;
    std::vector<hipGraphNode *> deps;
    size_t index = 0;
};

struct ihipGraph {
    std::vector<std::unique_ptr<hipGraphNode>> nodes;
};

struct hipGraphExec {
    struct N {
        int32_t kid;
        std::vector<uint8_t> args;
        uint32_t np;
    };
    std::vector<N> nodes;
};

namespace {

std::set<hipStream_t> g_streams;
std::set<hipEvent_t> g_events;
std::set<hipGraph_t> g_graphs;
std::map<hipGraphExec_t, std::shared_ptr<hipGraphExec>> g_execs;

void (*g_hook)(int32_t kid, const void *args) = nullptr;

size_t args_size(int32_t kid)
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

// "function pointers" of the standalone kernels: one tag per task id
struct KernelTag {
    int32_t kid;
};
KernelTag g_tags[ACS_K_COUNT];

void run_kernel(int32_t kid, const std::vector<uint8_t> &a, uint32_t np)
{
    if (np == 0) die("kernel launched with no workgroups");
    switch (kid) {
    case ACS_K_NOP: break;
    case ACS_K_COPY: {
        acs_args_copy c;
        memcpy(&c, a.data(), sizeof(c));
        memcpy(c.dst, c.src, (size_t)c.bytes);
        break;
    }
    case ACS_K_SIGNAL: {
        acs_args_signal s;
        memcpy(&s, a.data(), sizeof(s));
        __atomic_store_n(s.addr, s.value, __ATOMIC_RELEASE);
        break;
    }
    default:
        if (g_hook) g_hook(kid, a.data());
        break;
    }
}

bool live_stream(hipStream_t s) { return g_streams.count(s) != 0; }

// runs one queued operation of s; false if none
bool step(hipStream_t s)
{
    if (s->q.empty()) return false;
    Op op = std::move(s->q.front());
    s->q.pop_front();
    op();
    return true;
}

void drain(hipStream_t s)
{
    while (step(s)) {
    }
}

}  // namespace

extern "C" void fake_hip_set_kernel_hook(void (*hook)(int32_t, const void *)) { g_hook = hook; }

// every object still alive (a leak check for the tests)
extern "C" void fake_hip_counts(int64_t *out)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    out[0] = (int64_t)g_streams.size();
    out[1] = (int64_t)g_events.size();
    out[2] = (int64_t)g_graphs.size();
    out[3] = (int64_t)g_execs.size();
    out[4] = (int64_t)g_dev.size();
    out[5] = (int64_t)g_host.size();
}

hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidValue; }

hipError_t hipDeviceGetAttribute(int *value, hipDeviceAttribute_t attr, int device)
{
    if (device != 0) return hipErrorInvalidValue;
    *value = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 100000;
    return hipSuccess;
}

hipError_t hipRuntimeGetVersion(int *version)
{
    *version = 0;
    return hipSuccess;
}

hipError_t hipDeviceSynchronize(void)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    for (bool any = true; any;) {
        any = false;
        for (hipStream_t s : g_streams) any |= step(s);
    }
    return hipSuccess;
}

const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "fake HIP error"; }

hipError_t hipMalloc(void **p, size_t bytes)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *p = aligned_alloc(256, (bytes + 255) & ~size_t(255));
    if (!*p) return hipErrorOutOfMemory;
    g_dev.insert(*p);
    return hipSuccess;
}

hipError_t hipFree(void *p)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!p) return hipSuccess;
    if (!g_dev.erase(p)) die("hipFree of a pointer hipMalloc did not return");
    free(p);
    return hipSuccess;
}

hipError_t hipHostMalloc(void **p, size_t bytes, unsigned int)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *p = aligned_alloc(256, (bytes + 255) & ~size_t(255));
    if (!*p) return hipErrorOutOfMemory;
    g_host.insert(*p);
    return hipSuccess;
}

hipError_t hipHostFree(void *p)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!p) return hipSuccess;
    if (!g_host.erase(p)) die("hipHostFree of a pointer hipHostMalloc did not return");
    // freeing pinned memory waits for the device, as the runtime does
    hipDeviceSynchronize();
    free(p);
    return hipSuccess;
}

hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind)
{
    hipDeviceSynchronize();
    memcpy(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemset(void *dst, int value, size_t bytes)
{
    hipDeviceSynchronize();
    memset(dst, value, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *s = new ihipStream_t();
    g_streams.insert(*s);
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!live_stream(s)) die("hipStreamDestroy of a destroyed or unknown stream");
    drain(s);   // the runtime finishes a destroyed stream's work
    for (hipEvent_t e : g_events)
        if (e->stream == s) e->stream = nullptr;
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}

hipError_t hipStreamGetDevice(hipStream_t s, hipDevice_t *device)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!live_stream(s)) die("hipStreamGetDevice of a destroyed or unknown stream");
    *device = 0;
    return hipSuccess;
}

hipError_t hipStreamQuery(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!live_stream(s)) die("hipStreamQuery of a destroyed or unknown stream");
    for (uint64_t k = rnd() % 3; k > 0 && step(s); k--) {
    }
    return s->q.empty() ? hipSuccess : hipErrorNotReady;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!live_stream(s)) die("hipStreamSynchronize of a destroyed or unknown stream");
    drain(s);
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int flags)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *e = new ihipEvent_t();
    (*e)->flags = flags;
    g_events.insert(*e);
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_events.count(e)) die("hipEventDestroy of a destroyed or unknown event");
    // a pending record keeps running on its stream; it must not touch the event
    if (e->pending && e->stream) drain(e->stream);
    g_events.erase(e);
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_events.count(e)) die("hipEventRecord of a destroyed or unknown event");
    if (!live_stream(s)) die("hipEventRecord on a destroyed or unknown stream");
    if (e->pending && e->stream) drain(e->stream);   // a re-record supersedes the pending one
    e->pending = true;
    e->stream = s;
    s->q.push_back([e] {
        if (!g_events.count(e)) die("an event was freed under its pending record");
        e->pending = false;
        e->t = ++g_clock;
    });
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_events.count(e)) die("hipEventQuery of a destroyed or unknown event");
    if (e->pending && e->stream && rnd() % 2) step(e->stream);
    return e->pending ? hipErrorNotReady : hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_events.count(e)) die("hipEventSynchronize of a destroyed or unknown event");
    while (e->pending && e->stream && step(e->stream)) {
    }
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_events.count(a) || !g_events.count(b)) die("hipEventElapsedTime of a destroyed or unknown event");
    if ((a->flags | b->flags) & hipEventDisableTiming) return hipErrorInvalidValue;
    if (a->pending || b->pending) return hipErrorNotReady;
    *ms = (float)((double)b->t - (double)a->t) * 1e-3f;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!live_stream(s)) die("hipStreamWaitEvent on a destroyed or unknown stream");
    if (!g_events.count(e)) die("hipStreamWaitEvent on a destroyed or unknown event");
    if (!e->pending) return hipSuccess;   // the wait is on the event's state at the time of the call
    hipStream_t src = e->stream;
    const uint64_t t_before = e->t;
    s->q.push_back([e, src, t_before] {
        // drive the producer until the awaited record has run
        if (g_events.count(e)) {
            while (e->pending && e->t == t_before && live_stream(src) && step(src)) {
            }
        }
    });
    return hipSuccess;
}

hipError_t hipGraphCreate(hipGraph_t *g, unsigned int)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    *g = new ihipGraph();
    g_graphs.insert(*g);
    return hipSuccess;
}

hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *deps, size_t n_deps,
                                 const hipKernelNodeParams *p)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_graphs.count(g)) die("hipGraphAddKernelNode on a destroyed or unknown graph");
    const KernelTag *tag = static_cast<const KernelTag *>(p->func);
    if (tag < g_tags || tag >= g_tags + ACS_K_COUNT) die("kernel node with an unknown function");
    if (p->gridDim.x == 0 || p->blockDim.x != ACS_BLOCK || !p->kernelParams) die("bad kernel node parameters");
    auto n = std::make_unique<hipGraphNode>();
    n->kid = tag->kid;
    const size_t sz = args_size(tag->kid);
    n->args.resize(sz);
    memcpy(n->args.data(), p->kernelParams[0], sz);    // the runtime copies each argument now
    memcpy(&n->np, p->kernelParams[1], sizeof(uint32_t));
    if (n->np != p->gridDim.x) die("kernel node: piece count differs from the grid");
    for (size_t i = 0; i < n_deps; i++) {
        bool found = false;
        for (auto &m : g->nodes) found |= m.get() == deps[i];
        if (!found) die("kernel node depends on a node of another graph");
        n->deps.push_back(deps[i]);
    }
    n->index = g->nodes.size();
    *node = n.get();
    g->nodes.push_back(std::move(n));
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *, char *, size_t)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_graphs.count(g)) die("hipGraphInstantiate of a destroyed or unknown graph");
    auto x = std::make_shared<hipGraphExec>();
    for (auto &n : g->nodes) {
        for (hipGraphNode *d : n->deps)
            if (d->index >= n->index) die("graph nodes are not in a topological order");
        x->nodes.push_back({n->kid, n->args, n->np});
    }
    *exec = x.get();
    g_execs[*exec] = x;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    auto it = g_execs.find(exec);
    if (it == g_execs.end()) die("hipGraphLaunch of a destroyed or unknown executable graph");
    if (!live_stream(s)) die("hipGraphLaunch on a destroyed or unknown stream");
    std::shared_ptr<hipGraphExec> x = it->second;   // a launched graph outlives its destruction
    s->q.push_back([x] {
        for (auto &n : x->nodes) run_kernel(n.kid, n.args, n.np);
    });
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_execs.erase(exec)) die("hipGraphExecDestroy of a destroyed or unknown executable graph");
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (!g_graphs.erase(g)) die("hipGraphDestroy of a destroyed or unknown graph");
    delete g;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// the device-code entry points of launch.hpp
// ---------------------------------------------------------------------------
namespace acs {

hipError_t launch_task(int32_t kid, const void *args, uint32_t npieces, hipStream_t stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    const size_t sz = args_size(kid);
    if (sz == 0 || npieces == 0) return hipErrorInvalidValue;
    if (!live_stream(stream)) die("kernel launched on a destroyed or unknown stream");
    std::vector<uint8_t> a(sz);
    memcpy(a.data(), args, sz);   // launch arguments are copied at launch
    stream->q.push_back([kid, a, npieces] { run_kernel(kid, a, npieces); });
    return hipSuccess;
}

const void *task_kernel(int32_t kid)
{
    if (kid < 0 || kid >= ACS_K_COUNT || args_size(kid) == 0) return nullptr;
    g_tags[kid].kid = kid;
    return &g_tags[kid];
}

hipError_t launch_multi(const MultiParams &p, hipStream_t stream)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    if (p.n == 0 || p.n > (uint32_t)kMultiMax || p.total == 0) return hipErrorInvalidValue;
    if (!live_stream(stream)) die("kernel launched on a destroyed or unknown stream");
    std::vector<std::pair<int32_t, std::vector<uint8_t>>> ts;
    std::vector<uint32_t> nps;
    for (uint32_t i = 0; i < p.n; i++) {
        const size_t sz = args_size(p.t[i].kid);
        if (sz == 0 || p.t[i].np == 0) return hipErrorInvalidValue;
        ts.emplace_back(p.t[i].kid, std::vector<uint8_t>(p.t[i].args, p.t[i].args + sz));
        nps.push_back(p.t[i].np);
    }
    stream->q.push_back([ts, nps] {
        for (size_t i = 0; i < ts.size(); i++) run_kernel(ts[i].first, ts[i].second, nps[i]);
    });
    return hipSuccess;
}

// the persistent kernel has no host stand-in: the device path cannot start
hipError_t launch_persistent(const DevParams &, int32_t, hipStream_t) { return hipErrorInvalidValue; }

hipError_t persistent_blocks_per_cu(int32_t, int32_t *blocks)
{
    *blocks = 2;
    return hipSuccess;
}

hipError_t persistent_lds_bytes(int32_t, int32_t *bytes)
{
    *bytes = 0;
    return hipSuccess;
}

// no device state either: a window without allocation cannot start
hipError_t static_state(int32_t, DevState **) { return hipErrorInvalidValue; }

hipError_t clear_state(DevState *, hipStream_t) { return hipErrorInvalidValue; }

}  // namespace acs
