// Graph capture of a repeating task graph (acs_graph_*): the recorded
// kernels become nodes of one HIP graph whose edges are the read/write
// conflicts among them, replayed without a window.
#include <hip/hip_runtime_api.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

struct acs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t stream = nullptr;
    int32_t device = 0;
    int64_t n_kernels = 0, n_edges = 0;
};

namespace {

int graph_fail(hipError_t e, const char *what)
{
    acs::set_error(ACS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return ACS_EDEVICE;
}

// Launch streams are kept for reuse once their graph is destroyed: a graph
// rebuilt for every input then costs its construction, not a stream.
std::mutex g_pool_mu;
std::map<int32_t, std::vector<hipStream_t>> g_stream_pool;

hipError_t take_stream(int32_t device, hipStream_t *out)
{
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto &v = g_stream_pool[device];
        if (!v.empty()) {
            *out = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
}

void give_stream(int32_t device, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_stream_pool[device].push_back(s);
}

void destroy_parts(acs_graph *g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->stream) give_stream(g->device, g->stream);
    g->exec = nullptr;
    g->graph = nullptr;
    g->stream = nullptr;
}

}  // namespace

extern "C" {

int acs_graph_begin(acs_window *w)
{
    if (!w) {
        acs::set_error(ACS_EINVAL, "null window");
        return ACS_EINVAL;
    }
    if (w->recording || w->stopped) {
        acs::set_error(ACS_ESTATE, w->recording ? "already recording" : "window was stopped");
        return ACS_ESTATE;
    }
    w->recording = true;
    w->recorded.clear();
    return ACS_OK;
}

int acs_graph_end(acs_window *w, acs_graph **out)
{
    if (!w || !out) {
        acs::set_error(ACS_EINVAL, "null argument");
        return ACS_EINVAL;
    }
    if (!w->recording) {
        acs::set_error(ACS_ESTATE, "not recording");
        return ACS_ESTATE;
    }
    w->recording = false;
    const std::vector<acs::Desc> ks = std::move(w->recorded);
    w->recorded.clear();
    const size_t n = ks.size();
    if (n == 0) {
        acs::set_error(ACS_EINVAL, "nothing was recorded");
        return ACS_EINVAL;
    }
    // Dependencies: j after every earlier conflicting i, minus the edges that
    // a kept edge already implies (i is an ancestor of some kept parent).
    const size_t words = (n + 63) / 64;
    std::vector<uint64_t> anc(n * words, 0);   // anc[j]: every ancestor of j
    std::vector<std::vector<size_t>> parents(n);
    int64_t edges = 0;
    for (size_t j = 0; j < n; j++) {
        uint64_t *aj = &anc[j * words];
        for (size_t ii = j; ii-- > 0;) {   // newest first: a nearer conflict covers older ones it depends on
            if ((aj[ii / 64] >> (ii % 64)) & 1ull) continue;
            if (!acs::descs_conflict(ks[ii], ks[j], nullptr)) continue;
            parents[j].push_back(ii);
            edges++;
            aj[ii / 64] |= 1ull << (ii % 64);
            const uint64_t *ai = &anc[ii * words];
            for (size_t q = 0; q < words; q++) aj[q] |= ai[q];
        }
    }
    acs_graph *g = new (std::nothrow) acs_graph();
    if (!g) {
        acs::set_error(ACS_ENOMEM, "out of memory");
        return ACS_ENOMEM;
    }
    hipError_t e;
    if ((e = hipSetDevice(w->cfg.device)) != hipSuccess || (e = hipGraphCreate(&g->graph, 0)) != hipSuccess) {
        delete g;
        return graph_fail(e, "hipGraphCreate");
    }
    std::vector<hipGraphNode_t> nodes(n, nullptr);
    std::vector<hipGraphNode_t> deps;
    for (size_t j = 0; j < n; j++) {
        const acs::Desc &d = ks[j];
        const void *fn = acs::task_kernel(d.kid);
        if (!fn) {
            destroy_parts(g);
            delete g;
            acs::set_error(ACS_EINVAL, "task has no standalone kernel");
            return ACS_EINVAL;
        }
        uint32_t np = d.npieces;
        void *params[2] = {const_cast<uint8_t *>(d.args), &np};   // copied when the node is added
        hipKernelNodeParams kp = {};
        kp.func = const_cast<void *>(fn);
        kp.gridDim = dim3(np);
        kp.blockDim = dim3(ACS_BLOCK);
        kp.sharedMemBytes = 0;
        kp.kernelParams = params;
        kp.extra = nullptr;
        deps.clear();
        for (size_t i : parents[j]) deps.push_back(nodes[i]);
        if ((e = hipGraphAddKernelNode(&nodes[j], g->graph, deps.empty() ? nullptr : deps.data(), deps.size(), &kp)) !=
            hipSuccess) {
            destroy_parts(g);
            delete g;
            return graph_fail(e, "hipGraphAddKernelNode");
        }
    }
    g->device = w->cfg.device;
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess ||
        (e = take_stream(g->device, &g->stream)) != hipSuccess) {
        destroy_parts(g);
        delete g;
        return graph_fail(e, "hipGraphInstantiate");
    }
    g->n_kernels = (int64_t)n;
    g->n_edges = edges;
    *out = g;
    return ACS_OK;
}

int acs_graph_launch(acs_graph *g)
{
    if (!g || !g->exec) {
        acs::set_error(ACS_EINVAL, "null graph");
        return ACS_EINVAL;
    }
    const hipError_t e = hipGraphLaunch(g->exec, g->stream);
    return e == hipSuccess ? ACS_OK : graph_fail(e, "hipGraphLaunch");
}

int acs_graph_sync(acs_graph *g)
{
    if (!g || !g->stream) {
        acs::set_error(ACS_EINVAL, "null graph");
        return ACS_EINVAL;
    }
    const hipError_t e = hipStreamSynchronize(g->stream);
    return e == hipSuccess ? ACS_OK : graph_fail(e, "hipStreamSynchronize");
}

int acs_graph_info(const acs_graph *g, int64_t *n_kernels, int64_t *n_edges)
{
    if (!g) {
        acs::set_error(ACS_EINVAL, "null graph");
        return ACS_EINVAL;
    }
    if (n_kernels) *n_kernels = g->n_kernels;
    if (n_edges) *n_edges = g->n_edges;
    return ACS_OK;
}

int acs_graph_destroy(acs_graph *g)
{
    if (!g) return ACS_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    destroy_parts(g);
    delete g;
    return ACS_OK;
}

}  // extern "C"
