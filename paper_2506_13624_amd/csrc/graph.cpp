// Stream capture into HIP graphs: a caller records a sequence of the
// library's asynchronous calls once (for example shift -> warm solve, or
// network -> scatter -> guarded solve) and replays it with one launch.
#include <hip/hip_runtime.h>

#include "bmpc_internal.hpp"

struct bmpc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace bmpc;

extern "C" {

BMPC_API bmpc_status bmpc_graph_begin(void* stream)
{
    if (!stream) return fail(BMPC_ERR_INVALID_ARG, "capture needs a created stream, not the default stream");
    BMPC_HIP_TRY(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_graph_end(void* stream, bmpc_graph** out)
{
    if (!stream || !out) return fail(BMPC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    hipGraph_t g = nullptr;
    BMPC_HIP_TRY(hipStreamEndCapture((hipStream_t)stream, &g));
    if (!g) return fail(BMPC_ERR_HIP, "capture produced no graph");
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(BMPC_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(err));
    }
    auto* r = new bmpc_graph();
    r->graph = g;
    r->exec = e;
    *out = r;
    return BMPC_OK;
}

BMPC_API bmpc_status bmpc_graph_launch(bmpc_graph* g, void* stream)
{
    if (!g) return fail(BMPC_ERR_INVALID_ARG, "graph is NULL");
    BMPC_HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return BMPC_OK;
}

BMPC_API void bmpc_graph_destroy(bmpc_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
