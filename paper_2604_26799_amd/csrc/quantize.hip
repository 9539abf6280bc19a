// Final group-wise quantization at a chosen bit allocation, and its inverse.
// Paper: section "Group-wise Attribute Quantization" (quantizer; the block
// minimum and maximum are stored for decoding) and section "Entropy
// Encoding" (those bounds are part of the metadata).
//
// Both kernels are HBM-bound: one workgroup per (channel, group) reads the
// group's values once for the minimum / maximum and keeps them in registers
// for the codes (up to 16 values per thread: groups beyond 16384 elements
// (1024 threads) or 2048 (256 threads) read them again, from L2); the
// dequantizer reads 2-byte codes and writes FP32 values.  The
// quantizer expression is the literal FP32 definition, so codes equal those
// of the sweep bit for bit.
#include <algorithm>

#include "common.h"

namespace mgs {
namespace {


__device__ __forceinline__ int clamp_bits(uint8_t b) { return b < 1 ? 1 : (b > 16 ? 16 : b); }

// One workgroup of QT threads per (channel, group), groups strided over the
// grid.  A batch is QT * QU consecutive elements of the group: every thread
// first issues its QU index loads, then its QU value loads, so that each
// thread has QU gathers in flight instead of one.  Groups of up to QT * QU
// elements stay in registers between the minimum / maximum and the codes.
template <int QT, int QU>
__global__ __launch_bounds__(QT) void quantize_kernel(const float* __restrict__ attr, int64_t ld,
                                                      int C, const int32_t* __restrict__ kept,
                                                      int64_t k, int G, int64_t ng,
                                                      const uint8_t* __restrict__ bw,
                                                      uint16_t* __restrict__ codes,
                                                      float* __restrict__ gmin,
                                                      float* __restrict__ gmax) {
    constexpr int CAP = QT * QU;
    __shared__ float smn[QT / MGS_WAVE], smx[QT / MGS_WAVE];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int64_t blk = blockIdx.x; blk < (int64_t)C * ng; blk += gridDim.x) {
        const int c = (int)(blk / ng);
        const int64_t g = blk - (int64_t)c * ng;
        const int64_t j0 = g * G;
        const int n = (int)std::min<int64_t>(G, k - j0);
        const float* row = attr + (int64_t)c * ld;
        const int32_t* J = kept + j0;
        float xr[QU];
        auto load = [&](int b0) {
            int32_t id[QU];
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int j = b0 + u * QT + tid;
                id[u] = j < n ? J[j] : 0;
            }
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int j = b0 + u * QT + tid;
                xr[u] = j < n ? row[id[u]] : 0.0f;
            }
        };
        float mn = INFINITY, mx = -INFINITY;
        for (int b0 = 0; b0 < n; b0 += CAP) {
            load(b0);
#pragma unroll
            for (int u = 0; u < QU; ++u)
                if (b0 + u * QT + tid < n) {
                    mn = fminf(mn, xr[u]);
                    mx = fmaxf(mx, xr[u]);
                }
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
        if (tid == 0) {
            gmin[blk] = mn;
            gmax[blk] = mx;
        }
        uint16_t* out = codes + (int64_t)c * k + j0;
        const float qmax = P - 1.0f;
        for (int b0 = 0; b0 < n; b0 += CAP) {
            if (n > CAP) load(b0);  // otherwise the group is still in registers
#pragma unroll
            for (int u = 0; u < QU; ++u) {
                const int j = b0 + u * QT + tid;
                if (j < n) {
                    uint16_t q = 0;
                    if (S != 0.0f) {
                        float t = xr[u] / S;
                        t = t + Z;
                        t = __builtin_amdgcn_fmed3f(t, 0.0f, qmax);
                        q = (uint16_t)__builtin_rintf(t);
                    }
                    out[j] = q;
                }
            }
        }
        __syncthreads();  // smn / smx are reused by the next group
    }
}

// Dequantizer: a workgroup takes one piece of DT * 8 codes of a group (so
// that a launch has many more workgroups than CUs even for few groups), and
// each thread 8 consecutive codes: one 16-byte load and two 16-byte stores
// when the piece starts on a multiple of 8 elements of the row and the
// buffers are 16-byte aligned (vec), element by element otherwise.
constexpr int DQ_PER = 8;
template <int DT>
__global__ __launch_bounds__(DT) void dequantize_kernel(const uint16_t* __restrict__ codes,
                                                        int64_t k, int C, int G, int64_t ng, int nchunk,
                                                        const uint8_t* __restrict__ bw,
                                                        const float* __restrict__ gmin,
                                                        const float* __restrict__ gmax,
                                                        float* __restrict__ out, int vec) {
    const int tid = threadIdx.x;
    const int64_t nblk = (int64_t)C * ng * nchunk;
    for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const int64_t grp = blk / nchunk;  // (channel, group), channel-major
        const int ch = (int)(blk - grp * nchunk);
        const int c = (int)(grp / ng);
        const int64_t g = grp - (int64_t)c * ng;
        const int64_t j0 = g * G + (int64_t)ch * DT * DQ_PER;
        const int64_t gend = std::min<int64_t>(k, (g + 1) * (int64_t)G);
        if (j0 >= gend) continue;
        const int m = (int)std::min<int64_t>(DT * DQ_PER, gend - j0);
        const float mn = gmin[grp], mx = gmax[grp];
        const int b = clamp_bits(bw[grp]);
        const float P = ldexpf(1.0f, b);
        const float R = mx - mn;
        const float S = R / P;
        float Z = 0.0f;
        if (S != 0.0f) {
            float r = mx / S;
            Z = __builtin_rintf(P - r);
        }
        auto deq = [&](uint32_t q) {
            float v = mn;
            if (S != 0.0f) {
                float d = (float)q - Z;
                v = d * S;
            }
            return v;
        };
        const int64_t off = (int64_t)c * k + j0;
        const int e0 = tid * DQ_PER;
        if (vec && (off % DQ_PER) == 0 && e0 + DQ_PER <= m) {
            const uint4 raw = *reinterpret_cast<const uint4*>(codes + off + e0);
            const uint32_t w[4] = {raw.x, raw.y, raw.z, raw.w};
            float v[DQ_PER];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[2 * i] = deq(w[i] & 0xFFFFu);
                v[2 * i + 1] = deq(w[i] >> 16);
            }
            float4* o4 = reinterpret_cast<float4*>(out + off + e0);
            o4[0] = make_float4(v[0], v[1], v[2], v[3]);
            o4[1] = make_float4(v[4], v[5], v[6], v[7]);
        } else {
#pragma unroll
            for (int i = 0; i < DQ_PER; ++i) {
                const int e = e0 + i;
                if (e < m) out[off + e] = deq(codes[off + e]);
            }
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
    // large groups: 1024 threads per group, 8 or 16 values per thread (a group
    // of up to 16384 is gathered once); small ones: 256 threads
    if (G > 8192)
        hipLaunchKernelGGL((mgs::quantize_kernel<1024, 16>), dim3((unsigned)blocks), dim3(1024), 0,
                           (hipStream_t)stream, d_attr, ld, C, d_kept, k, G, ng, d_bw, d_codes, d_gmin,
                           d_gmax);
    else if (G >= 4096)
        hipLaunchKernelGGL((mgs::quantize_kernel<1024, 8>), dim3((unsigned)blocks), dim3(1024), 0,
                           (hipStream_t)stream, d_attr, ld, C, d_kept, k, G, ng, d_bw, d_codes, d_gmin,
                           d_gmax);
    else
        hipLaunchKernelGGL((mgs::quantize_kernel<256, 8>), dim3((unsigned)blocks), dim3(256), 0,
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
    constexpr int DT = 256;
    const int nchunk = (G + DT * mgs::DQ_PER - 1) / (DT * mgs::DQ_PER);
    const int64_t blocks = std::min<int64_t>((int64_t)C * ng * nchunk, 1 << 20);
    const int vec = ((uintptr_t)d_codes % 16 == 0) && ((uintptr_t)d_out % 16 == 0);
    hipLaunchKernelGGL(mgs::dequantize_kernel<DT>, dim3((unsigned)blocks), dim3(DT), 0, (hipStream_t)stream,
                       d_codes, k, C, G, ng, nchunk, d_bw, d_gmin, d_gmax, d_out, vec);
    return mgs_last_launch();
}
