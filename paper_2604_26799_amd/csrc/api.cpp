// Status text, version and the device status word of a workspace.
#include <hip/hip_runtime.h>

#include "common.h"

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
