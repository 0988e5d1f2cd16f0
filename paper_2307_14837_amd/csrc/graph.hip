// HIP-graph capture of a sequence of library calls (a whole correction step,
// a batched step, a training step), so that a time loop replays the step
// with one launch of the executable graph instead of re-issuing each kernel.
#include "common.hpp"

struct dnnmg_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

using namespace dnnmg;

extern "C" int dnnmg_graph_capture_begin(void *stream) {
    if (!stream) return fail(DNNMG_ERR_ARG, "dnnmg_graph_capture_begin: the legacy default stream cannot be captured");
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing((hipStream_t)stream, &st);
    if (e != hipSuccess) return hip_check(e, "dnnmg_graph_capture_begin: hipStreamIsCapturing");
    if (st != hipStreamCaptureStatusNone)
        return fail(DNNMG_ERR_ARG, "dnnmg_graph_capture_begin: the stream is already capturing");
    return hip_check(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal),
                     "dnnmg_graph_capture_begin: hipStreamBeginCapture");
}

extern "C" int dnnmg_graph_capture_end(void *stream, dnnmg_graph **out) {
    if (!stream || !out) return fail(DNNMG_ERR_ARG, "dnnmg_graph_capture_end: NULL stream or output");
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_check(e, "dnnmg_graph_capture_end: hipStreamEndCapture");
    }
    if (!g) return fail(DNNMG_ERR_HIP, "dnnmg_graph_capture_end: the capture produced no graph");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_check(e, "dnnmg_graph_capture_end: hipGraphInstantiate");
    }
    *out = new dnnmg_graph{g, x};
    return DNNMG_OK;
}

extern "C" int dnnmg_graph_replay(const dnnmg_graph *graph, void *stream) {
    if (!graph) return fail(DNNMG_ERR_ARG, "dnnmg_graph_replay: NULL graph");
    return hip_check(hipGraphLaunch(graph->exec, (hipStream_t)stream), "dnnmg_graph_replay: hipGraphLaunch");
}

extern "C" int dnnmg_graph_destroy(dnnmg_graph *graph) {
    if (!graph) return DNNMG_OK;
    hipError_t e1 = hipGraphExecDestroy(graph->exec);
    hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    if (e1 != hipSuccess) return hip_check(e1, "dnnmg_graph_destroy: hipGraphExecDestroy");
    return hip_check(e2, "dnnmg_graph_destroy: hipGraphDestroy");
}
