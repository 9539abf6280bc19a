// Internal helpers shared by the libmgs HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mgs.h"

#define MGS_WAVE 64

// Status word layout at the start of every workspace.
struct mgs_status_block {
    uint32_t nonfinite;
    uint32_t pad0[15];
    uint32_t queue[16];  // tile counters of a persistent launch (one per XCD), reset with the status
    uint32_t pad[32];
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
// FP64 sum over the wavefront with DPP row shifts and row broadcasts (no LDS
// traffic); the fixed pattern makes the result deterministic.  Returns the
// total in every lane (read from lane 63).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_total_f64(double v) {
    v += dpp_f64<0x111, 0xF>(v);  // row_shr:1   (inclusive prefix within rows of 16)
    v += dpp_f64<0x112, 0xF>(v);  // row_shr:2
    v += dpp_f64<0x114, 0xF>(v);  // row_shr:4
    v += dpp_f64<0x118, 0xF>(v);  // row_shr:8   -> lane 15 of each row: row sum
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63: total
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}
// The same fixed pattern in FP32 (each step is one DPP add): for sums of
// nonnegative terms every step adds at most 2^-24 relative error, six in all.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, true));
}
__device__ __forceinline__ float wave_total_f32(float v) {
    v += dpp_f32<0x111, 0xF>(v);
    v += dpp_f32<0x112, 0xF>(v);
    v += dpp_f32<0x114, 0xF>(v);
    v += dpp_f32<0x118, 0xF>(v);
    v += dpp_f32<0x142, 0xA>(v);
    v += dpp_f32<0x143, 0xC>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
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
