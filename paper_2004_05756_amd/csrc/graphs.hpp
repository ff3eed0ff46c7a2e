// Kernel launches recorded into HIP graphs node by node (no stream capture), and the
// per-context cache of instantiated graphs keyed by every value baked into their
// kernel arguments.
#pragma once

#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_ext.h>

#include "internal.hpp"

namespace topo {

// Graph replays are on unless TOPO_NO_GRAPH is set (then every launch is direct, which
// is how the counter runs see each dispatch).
inline bool graphs_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("TOPO_NO_GRAPH");
        return !(e && e[0] && e[0] != '0');
    }();
    return on;
}

// Instantiated graphs a context keeps before it releases them all.
constexpr size_t kGraphCacheMax = 16;

// Where kernel launches go: directly onto a stream, or appended as kernel nodes (each
// depending on the previous one) to a graph under construction.  Graphs are built
// node by node rather than by stream capture, so that building one never interferes
// with launches that other threads make at the same time.  Argument types must match
// the kernel's parameters exactly.
struct LaunchSink {
    hipStream_t s = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t err = hipSuccess;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // kernel start / end stamps of the next launch
    template <typename... A>
    void operator()(const void* fn, dim3 grid, dim3 block, A... args) {
        void* ptrs[] = {(void*)&args...};
        hipError_t e;
        if (!graph) {
            if (ev0)
                e = hipExtLaunchKernel(fn, grid, block, ptrs, 0, s, ev0, ev1, 0);
            else
                e = hipLaunchKernel(fn, grid, block, ptrs, 0, s);
            ev0 = ev1 = nullptr;
        } else {
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(fn);
            kp.gridDim = grid;
            kp.blockDim = block;
            kp.sharedMemBytes = 0;
            kp.kernelParams = ptrs;
            kp.extra = nullptr;
            hipGraphNode_t node = nullptr;
            e = hipGraphAddKernelNode(&node, graph, last ? &last : nullptr, last ? 1 : 0, &kp);
            if (e == hipSuccess) last = node;
        }
        if (e != hipSuccess && err == hipSuccess) err = e;
    }
};

// Instantiated graph for `key`, built by build(L) on first use and cached in ctx.  When
// the cache is full every entry is released, after the stream `s` the graphs of this
// context run on has drained: a graph launched earlier in the same call (or an earlier
// call on s) may still be executing, and its kernel arguments live in the executable
// graph.  Calls of one context on other streams are ordered by the caller (a context's
// calls share its workspace), so they have finished too.
template <typename Build>
static int cached_graph(Ctx* ctx, const std::vector<uintptr_t>& key, Build build, hipGraphExec_t* out,
                        hipStream_t s) {
    auto it = ctx->graphs.find(key);
    if (it != ctx->graphs.end()) {
        *out = it->second.exec;
        return TOPO_OK;
    }
    if (ctx->graphs.size() >= kGraphCacheMax) {
        TOPO_HIP(hipStreamSynchronize(s));
        for (auto& kv : ctx->graphs) {
            (void)hipGraphExecDestroy(kv.second.exec);
            (void)hipGraphDestroy(kv.second.graph);
        }
        ctx->graphs.clear();
    }
    GraphEntry ge;
    TOPO_HIP(hipGraphCreate(&ge.graph, 0));
    LaunchSink L;
    L.graph = ge.graph;
    build(L);
    if (L.err != hipSuccess) {
        (void)hipGraphDestroy(ge.graph);
        return set_error(ctx, TOPO_EDEVICE, "graph construction failed: %s", hipGetErrorString(L.err));
    }
    const hipError_t e1 = hipGraphInstantiateWithFlags(&ge.exec, ge.graph, 0);
    if (e1 != hipSuccess) {
        (void)hipGraphDestroy(ge.graph);
        return set_error(ctx, TOPO_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e1));
    }
    ctx->graphs[key] = ge;
    *out = ge.exec;
    return TOPO_OK;
}

static void key_push_double(std::vector<uintptr_t>& key, double v) {
    uint64_t ib;
    std::memcpy(&ib, &v, sizeof ib);
    key.push_back((uintptr_t)ib);
}

}  // namespace topo
