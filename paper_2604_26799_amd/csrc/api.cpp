// Status text, version and the device status word of a workspace.
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/mgs.h"

extern "C" const char* mgs_strerror(int status) {
    switch (status) {
        case MGS_OK: return "ok";
        case MGS_EINVAL: return "invalid argument";
        case MGS_ENONFINITE: return "non-finite input";
        case MGS_EINFEASIBLE: return "infeasible: the budget is below the smallest allocation";
        case MGS_EDEVICE: return "HIP device or launch error";
        case MGS_EWORKSPACE: return "workspace missing or too small";
        case MGS_ELIMIT: return "exact ILP search exceeded its state limit";
        default: return "unknown status";
    }
}

extern "C" const char* mgs_version(void) { return "libmgs 0.1 (gfx950)"; }

extern "C" int mgs_status_fetch(const void* d_ws, void* stream) {
    if (!d_ws) return MGS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return MGS_EDEVICE;
    uint32_t flag = 0;
    if (hipMemcpy(&flag, d_ws, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return MGS_EDEVICE;
    return flag ? MGS_ENONFINITE : MGS_OK;
}

// Stream capture into an executable graph.  Thread-local capture mode: a
// call on this thread that is not capture-safe fails the capture instead of
// silently running outside it.
extern "C" int mgs_graph_begin(void* stream) {
    if (!stream) return MGS_EINVAL;
    return hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal) == hipSuccess
               ? MGS_OK
               : MGS_EDEVICE;
}

extern "C" int mgs_graph_end(void* stream, void** h_graph) {
    if (!stream || !h_graph) return MGS_EINVAL;
    *h_graph = nullptr;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture((hipStream_t)stream, &g) != hipSuccess || !g) return MGS_EDEVICE;
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess || !exec) return MGS_EDEVICE;
    *h_graph = (void*)exec;
    return MGS_OK;
}

extern "C" int mgs_graph_launch(void* graph, void* stream) {
    if (!graph) return MGS_EINVAL;
    return hipGraphLaunch((hipGraphExec_t)graph, (hipStream_t)stream) == hipSuccess ? MGS_OK
                                                                                      : MGS_EDEVICE;
}

extern "C" int mgs_graph_destroy(void* graph) {
    if (!graph) return MGS_EINVAL;
    return hipGraphExecDestroy((hipGraphExec_t)graph) == hipSuccess ? MGS_OK : MGS_EDEVICE;
}
