// batch.cpp -- ragged batches captured into a HIP graph.
//
// The applies of a batch are independent (different meshes), so the capture
// forks the caller's stream into `lanes` streams, deals the descriptors out
// largest-first to the least-loaded lane (by algorithmic bytes), and joins the
// lanes back.  The graph then holds `lanes` independent chains of kernel
// nodes, which the runtime may run concurrently, and a replay costs one
// hipGraphLaunch.  All streams keep the default priority.
#include <algorithm>
#include <numeric>
#include <vector>

#include "fem.h"
#include "launch.hpp"

namespace fem {

int enqueue_desc(const fem_apply_desc &d, hipStream_t s);
double desc_bytes(const fem_apply_desc &d);

namespace {

struct BatchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
};

void release(BatchGraph *bg)
{
    // teardown: errors here leave nothing to recover, so they are not reported
    if (bg->exec) (void)hipGraphExecDestroy(bg->exec);
    if (bg->graph) (void)hipGraphDestroy(bg->graph);
    for (hipStream_t s : bg->side) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : bg->join) (void)hipEventDestroy(e);
    if (bg->fork) (void)hipEventDestroy(bg->fork);
    delete bg;
}

}  // namespace

int batch_graph_create(const fem_apply_desc *d, int n, int lanes, hipStream_t s, void **graph)
{
    auto *bg = new BatchGraph();
    bool ok = hipEventCreateWithFlags(&bg->fork, hipEventDisableTiming) == hipSuccess;
    for (int l = 1; l < lanes && ok; ++l) {
        hipStream_t side = nullptr;
        hipEvent_t ev = nullptr;
        ok = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess;
        if (ok) bg->side.push_back(side);
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) bg->join.push_back(ev);
    }
    if (!ok) {
        release(bg);
        return FEM_ERR_HIP;
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> bytes(n);
    for (int i = 0; i < n; ++i) bytes[i] = desc_bytes(d[i]);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return bytes[x] > bytes[y]; });

    int st = FEM_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        release(bg);
        return FEM_ERR_HIP;
    }
    ok = hipEventRecord(bg->fork, s) == hipSuccess;
    for (hipStream_t side : bg->side) ok = ok && hipStreamWaitEvent(side, bg->fork, 0) == hipSuccess;
    std::vector<double> load(lanes, 0.0);
    for (int idx : order) {
        if (!ok || st != FEM_OK) break;
        const int lane = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        st = enqueue_desc(d[idx], lane == 0 ? s : bg->side[lane - 1]);
        load[lane] += bytes[idx];
    }
    for (size_t l = 0; l < bg->side.size(); ++l) {
        ok = ok && hipEventRecord(bg->join[l], bg->side[l]) == hipSuccess;
        ok = ok && hipStreamWaitEvent(s, bg->join[l], 0) == hipSuccess;
    }
    const bool ended = hipStreamEndCapture(s, &bg->graph) == hipSuccess;
    if (!ok || !ended || st != FEM_OK) {
        release(bg);
        return st != FEM_OK ? st : FEM_ERR_HIP;
    }
    if (hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0) != hipSuccess) {
        release(bg);
        return FEM_ERR_HIP;
    }
    *graph = bg;
    return FEM_OK;
}

int batch_graph_launch(void *graph, hipStream_t s)
{
    auto *bg = static_cast<BatchGraph *>(graph);
    return hipGraphLaunch(bg->exec, s) == hipSuccess ? FEM_OK : FEM_ERR_HIP;
}

int batch_graph_destroy(void *graph)
{
    release(static_cast<BatchGraph *>(graph));
    return FEM_OK;
}

}  // namespace fem
