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

// The host search with a wait per ratio (ilp.cpp); here the waits are the
// caller's events, one per ratio, recorded after that ratio's table copies.
namespace mgs {
int search_tables(const mgs_sweep_desc* d, const double* h_err, const double* h_bits, int64_t budget_bits,
                  int32_t size_mode, int32_t threads, int32_t flags, int32_t* h_best_t, uint8_t* h_best_bits,
                  double* h_obj, int64_t* h_used, int32_t* h_status, int (*wait)(void*, int, int), void* wait_ctx);
}

static int wait_ratio_event(void* ctx, int t, int block) {
    hipEvent_t e = (hipEvent_t)((void* const*)ctx)[t];
    if (block) return hipEventSynchronize(e) == hipSuccess ? MGS_OK : MGS_EDEVICE;
    const hipError_t q = hipEventQuery(e);
    if (q == hipErrorNotReady) {
        (void)hipGetLastError();  // not an error: keep it out of the thread's last-error state
        return 1;
    }
    return q == hipSuccess ? MGS_OK : MGS_EDEVICE;
}

extern "C" int mgs_search_streamed(const mgs_sweep_desc* d, const double* h_err, const double* h_bits,
                                   int64_t budget_bits, int32_t size_mode, int32_t threads, int32_t flags,
                                   int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_used,
                                   int32_t* h_status, void* const* h_events) {
    if (!d || !h_events || d->T < 1 || d->T > MGS_MAX_RATIOS) return MGS_EINVAL;
    for (int t = 0; t < d->T; ++t)
        if (!h_events[t]) return MGS_EINVAL;
    return mgs::search_tables(d, h_err, h_bits, budget_bits, size_mode, threads, flags, h_best_t, h_best_bits,
                              h_obj, h_used, h_status, wait_ratio_event, (void*)h_events);
}
