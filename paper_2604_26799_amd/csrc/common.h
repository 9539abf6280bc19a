// Internal helpers shared by the libmgs HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mgs.h"

#define MGS_WAVE 64

// Status word layout at the start of every workspace.
struct mgs_status_block {
    uint32_t nonfinite;
    uint32_t pad[63];
};
static constexpr size_t MGS_STATUS_BYTES = sizeof(mgs_status_block);  // 256

static inline int mgs_hip_status(hipError_t e) { return e == hipSuccess ? MGS_OK : MGS_EDEVICE; }

static inline int mgs_last_launch() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MGS_OK : MGS_EDEVICE;
}

static inline size_t mgs_align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Wavefront reductions (64 lanes), butterfly via cross-lane shuffles.  Every
// lane ends with the full result; the combination order is fixed, so the
// result is deterministic.
__device__ __forceinline__ float wave_min_f32(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, MGS_WAVE));
    return v;
}
__device__ __forceinline__ float wave_max_f32(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, MGS_WAVE));
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = v + __shfl_xor(v, o, MGS_WAVE);
    return v;
}
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, MGS_WAVE);
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, MGS_WAVE);
    return v;
}

__device__ __forceinline__ bool finite_f32(float x) { return __builtin_isfinite(x); }

// Fill kernel used instead of memset so the calls stay graph-capturable.
template <typename T>
__global__ void mgs_fill_kernel(T* p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static inline int mgs_fill(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return MGS_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(mgs_fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return mgs_last_launch();
}
