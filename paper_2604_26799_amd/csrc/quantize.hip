// Final group-wise quantization at a chosen bit allocation, and its inverse.
// Paper: section "Group-wise Attribute Quantization" (quantizer; the block
// minimum and maximum are stored for decoding) and section "Entropy
// Encoding" (those bounds are part of the metadata).
//
// Both kernels are HBM-bound: one workgroup per (channel, group) reads the
// group's values once for the minimum / maximum and once more (from L2) for
// the codes; the dequantizer reads 2-byte codes and writes FP32 values.  The
// quantizer expression is the literal FP32 definition, so codes equal those
// of the sweep bit for bit.
#include <algorithm>

#include "common.h"

namespace mgs {
namespace {

constexpr int QT = 256;

__device__ __forceinline__ int clamp_bits(uint8_t b) { return b < 1 ? 1 : (b > 16 ? 16 : b); }

__global__ __launch_bounds__(QT) void quantize_kernel(const float* __restrict__ attr, int64_t ld,
                                                      int C, const int32_t* __restrict__ kept,
                                                      int64_t k, int G, int64_t ng,
                                                      const uint8_t* __restrict__ bw,
                                                      uint16_t* __restrict__ codes,
                                                      float* __restrict__ gmin,
                                                      float* __restrict__ gmax) {
    __shared__ float smn[QT / MGS_WAVE], smx[QT / MGS_WAVE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t blk = blockIdx.x; blk < (int64_t)C * ng; blk += gridDim.x) {
        const int c = (int)(blk / ng);
        const int64_t g = blk - (int64_t)c * ng;
        const int64_t j0 = g * G;
        const int n = (int)std::min<int64_t>(G, k - j0);
        const float* row = attr + (int64_t)c * ld;
        const int32_t* J = kept + j0;
        float mn = INFINITY, mx = -INFINITY;
        for (int j = threadIdx.x; j < n; j += QT) {
            float x = row[J[j]];
            mn = fminf(mn, x);
            mx = fmaxf(mx, x);
        }
        mn = wave_min_f32(mn);
        mx = wave_max_f32(mx);
        if (lane == 0) {
            smn[wave] = mn;
            smx[wave] = mx;
        }
        __syncthreads();
        mn = smn[0];
        mx = smx[0];
#pragma unroll
        for (int w = 1; w < QT / MGS_WAVE; ++w) {
            mn = fminf(mn, smn[w]);
            mx = fmaxf(mx, smx[w]);
        }
        const int b = clamp_bits(bw[blk]);
        const float P = ldexpf(1.0f, b);
        const float R = mx - mn;
        const float S = R / P;
        float Z = 0.0f;
        if (S != 0.0f) {
            float r = mx / S;
            Z = __builtin_rintf(P - r);
        }
        if (threadIdx.x == 0) {
            gmin[blk] = mn;
            gmax[blk] = mx;
        }
        uint16_t* out = codes + (int64_t)c * k + j0;
        const float qmax = P - 1.0f;
        for (int j = threadIdx.x; j < n; j += QT) {
            uint16_t q = 0;
            if (S != 0.0f) {
                float x = row[J[j]];
                float t = x / S;
                t = t + Z;
                t = __builtin_amdgcn_fmed3f(t, 0.0f, qmax);
                q = (uint16_t)__builtin_rintf(t);
            }
            out[j] = q;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(QT) void dequantize_kernel(const uint16_t* __restrict__ codes,
                                                        int64_t k, int C, int G, int64_t ng,
                                                        const uint8_t* __restrict__ bw,
                                                        const float* __restrict__ gmin,
                                                        const float* __restrict__ gmax,
                                                        float* __restrict__ out) {
    for (int64_t blk = blockIdx.x; blk < (int64_t)C * ng; blk += gridDim.x) {
        const int c = (int)(blk / ng);
        const int64_t g = blk - (int64_t)c * ng;
        const int64_t j0 = g * G;
        const int n = (int)std::min<int64_t>(G, k - j0);
        const float mn = gmin[blk], mx = gmax[blk];
        const int b = clamp_bits(bw[blk]);
        const float P = ldexpf(1.0f, b);
        const float R = mx - mn;
        const float S = R / P;
        float Z = 0.0f;
        if (S != 0.0f) {
            float r = mx / S;
            Z = __builtin_rintf(P - r);
        }
        const uint16_t* q = codes + (int64_t)c * k + j0;
        float* o = out + (int64_t)c * k + j0;
        for (int j = threadIdx.x; j < n; j += QT) {
            float v = mn;
            if (S != 0.0f) {
                float d = (float)q[j] - Z;
                v = d * S;
            }
            o[j] = v;
        }
    }
}

}  // namespace
}  // namespace mgs

extern "C" int mgs_quantize(const float* d_attr, int64_t ld, int32_t C, const int32_t* d_kept,
                            int64_t k, int32_t G, const uint8_t* d_bw, uint16_t* d_codes,
                            float* d_gmin, float* d_gmax, void* stream) {
    if (C < 1 || k < 0 || G < 1 || G > MGS_MAX_GROUP || ld < 0) return MGS_EINVAL;
    if (k == 0) return MGS_OK;
    if (!d_attr || !d_kept || !d_bw || !d_codes || !d_gmin || !d_gmax) return MGS_EINVAL;
    const int64_t ng = (k + G - 1) / G;
    const int64_t blocks = std::min<int64_t>((int64_t)C * ng, 1 << 20);
    hipLaunchKernelGGL(mgs::quantize_kernel, dim3((unsigned)blocks), dim3(mgs::QT), 0,
                       (hipStream_t)stream, d_attr, ld, C, d_kept, k, G, ng, d_bw, d_codes, d_gmin,
                       d_gmax);
    return mgs_last_launch();
}

extern "C" int mgs_dequantize(const uint16_t* d_codes, int64_t k, int32_t C, int32_t G,
                              const uint8_t* d_bw, const float* d_gmin, const float* d_gmax,
                              float* d_out, void* stream) {
    if (C < 1 || k < 0 || G < 1 || G > MGS_MAX_GROUP) return MGS_EINVAL;
    if (k == 0) return MGS_OK;
    if (!d_codes || !d_bw || !d_gmin || !d_gmax || !d_out) return MGS_EINVAL;
    const int64_t ng = (k + G - 1) / G;
    const int64_t blocks = std::min<int64_t>((int64_t)C * ng, 1 << 20);
    hipLaunchKernelGGL(mgs::dequantize_kernel, dim3((unsigned)blocks), dim3(mgs::QT), 0,
                       (hipStream_t)stream, d_codes, k, C, G, ng, d_bw, d_gmin, d_gmax, d_out);
    return mgs_last_launch();
}
