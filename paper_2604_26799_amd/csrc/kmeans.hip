// One iteration of mini-batch k-means around the nearest-codeword
// assignment.  Paper: section "Attribute Transformation", paragraph
// "Clustering 1+D SH Coefficients" -- the codebook of the higher-degree SH
// vectors is refined by a batched clustering strategy (Sculley's web-scale
// k-means) over several iterations.
//
// Per iteration, on a batch of sample rows chosen by the caller:
//   1. every batch row goes to its nearest center (the exact rule of
//      mgs_vq_assign: FP64 distance, ties to the smaller index);
//   2. center j, which has absorbed v_j samples so far and gets n_j > 0 rows
//      of this batch, moves to the running mean of all of them:
//        c_j <- (v_j c_j + sum of its batch rows) / (v_j + n_j),  v_j += n_j.
// Sculley's per-sample update (v += 1, eta = 1 / v, c <- (1 - eta) c + eta x,
// applied to the batch's rows in order) reaches the same mean.  The sum of a
// center's rows is taken in FP64 in batch order: the batch positions are
// sorted by center with a stable radix sort (rocPRIM), so each center's rows
// form one run in batch order, and one wave per center adds its run
// sequentially (lane d adds dimension d).  The result, rounded to FP32 once,
// is therefore the same on every run, bit for bit.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"

namespace mgs {
namespace {

struct KmArgs {
    const float* x;
    const int64_t* batch;
    float* xb;          // [B][D] gathered batch rows
    int32_t* assign;    // [B]
    uint32_t* keys;     // [B] sort keys: the center, K for rows without one
    uint32_t* keys_s;   // [B] the keys sorted
    int32_t* pos;       // [B] batch positions 0 .. B-1
    int32_t* pos_s;     // [B] batch positions in center order (stable: batch order within a center)
    float* cb;          // [K][D] centers (in place)
    int64_t* counts;    // [K] samples absorbed so far
    mgs_status_block* status;
    int64_t N, B;
    int32_t D, K;
};

// Batch rows into a contiguous block (one thread per value); an index
// outside [0, N) raises the status flag and gathers zeros.
__global__ void km_gather_kernel(KmArgs a) {
    const int64_t total = a.B * a.D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / a.D;
        const int d = (int)(i - r * a.D);
        const int64_t src = a.batch[r];
        float v = 0.0f;
        if (src >= 0 && src < a.N) v = a.x[src * a.D + d];
        else if (d == 0) atomicOr(&a.status->nonfinite, 2u);
        a.xb[i] = v;
    }
}

// Sort keys and batch positions of the batch rows.
__global__ void km_keys_kernel(KmArgs a) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.B;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int j = a.assign[r];
        a.keys[r] = (unsigned)j < (unsigned)a.K ? (uint32_t)j : (uint32_t)a.K;
        a.pos[r] = (int32_t)r;
    }
}

// First index of the sorted keys that is >= key.
__device__ __forceinline__ int64_t lower_bound_u32(const uint32_t* k, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (k[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One wave per center: the run of its rows in the sorted order, summed in
// batch order in FP64 (lane d: dimension d), then the running-mean update
// c <- (v c + sum) / (v + n) and v += n.  Centers without rows keep their
// value and count.
__global__ void km_center_kernel(KmArgs a) {
    const int lane = threadIdx.x & (MGS_WAVE - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / MGS_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / MGS_WAVE;
    for (int64_t j = wave; j < a.K; j += nwaves) {
        const int64_t lo = lower_bound_u32(a.keys_s, a.B, (uint32_t)j);
        const int64_t hi = lower_bound_u32(a.keys_s, a.B, (uint32_t)j + 1u);
        const int64_t n = hi - lo;
        if (n == 0) continue;
        const int64_t v = a.counts[j];
        if (lane < a.D) {
            const float* xd = a.xb + lane;
            double s = 0.0;
            int64_t i = lo;
            for (; i + 4 <= hi; i += 4) {  // four rows' loads in flight, added in order
                const float v0 = xd[(int64_t)a.pos_s[i] * a.D];
                const float v1 = xd[(int64_t)a.pos_s[i + 1] * a.D];
                const float v2 = xd[(int64_t)a.pos_s[i + 2] * a.D];
                const float v3 = xd[(int64_t)a.pos_s[i + 3] * a.D];
                s += (double)v0;
                s += (double)v1;
                s += (double)v2;
                s += (double)v3;
            }
            for (; i < hi; ++i) s += (double)xd[(int64_t)a.pos_s[i] * a.D];
            float* c = a.cb + j * a.D + lane;
            *c = (float)(((double)v * (double)*c + s) / (double)(v + n));
        }
        if (lane == 0) a.counts[j] = v + n;
    }
}

// The assignment's status word (non-finite rows or centers) into this call's.
__global__ void km_status_kernel(const mgs_status_block* vq, mgs_status_block* own) {
    if (threadIdx.x == 0 && vq->nonfinite) atomicOr(&own->nonfinite, vq->nonfinite);
}

struct KmLayout {
    size_t xb, assign, keys, keys_s, pos, pos_s, sort, sort_bytes, vq, total;
};

// Key bits of the sort: enough for the keys 0 .. K (K marks rows without a center).
int km_key_bits(int32_t K) {
    int bits = 1;
    while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)K) ++bits;
    return bits;
}

KmLayout km_layout(int64_t B, int32_t D, int32_t K) {
    KmLayout L;
    const size_t b = (size_t)std::max<int64_t>(B, 1);
    size_t o = MGS_STATUS_BYTES;
    L.xb = o;
    o += mgs_align_up(sizeof(float) * b * D, 256);
    L.assign = o;
    o += mgs_align_up(sizeof(int32_t) * b, 256);
    L.keys = o;
    o += mgs_align_up(sizeof(uint32_t) * b, 256);
    L.keys_s = o;
    o += mgs_align_up(sizeof(uint32_t) * b, 256);
    L.pos = o;
    o += mgs_align_up(sizeof(int32_t) * b, 256);
    L.pos_s = o;
    o += mgs_align_up(sizeof(int32_t) * b, 256);
    // temporary storage of the radix sort (a size query: no device work)
    L.sort_bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, L.sort_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                    (const int32_t*)nullptr, (int32_t*)nullptr, (unsigned)b, 0,
                                    km_key_bits(K));
    L.sort = o;
    o += mgs_align_up(std::max<size_t>(L.sort_bytes, 1), 256);
    L.vq = o;
    o += mgs_align_up(mgs_vq_assign_ws_bytes(B, D, K), 256);
    L.total = o;
    return L;
}

unsigned km_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

}  // namespace
}  // namespace mgs

extern "C" size_t mgs_kmeans_step_ws_bytes(int64_t B, int32_t D, int32_t K) {
    if (B < 0 || D < 1 || D > MGS_MAX_VQ_DIM || K < 1 || K > (1 << 30)) return 0;
    return mgs::km_layout(B, D, K).total;
}

extern "C" int mgs_kmeans_step(const float* d_x, int64_t N, int32_t D, const int64_t* d_batch, int64_t B,
                               float* d_cb, int32_t K, int64_t* d_counts, int32_t* d_assign, void* d_ws,
                               size_t ws_bytes, void* stream) {
    using namespace mgs;
    if (N < 0 || B < 0 || B >= ((int64_t)1 << 31) || D < 1 || D > MGS_MAX_VQ_DIM || K < 1 || K > (1 << 30) ||
        !d_cb ||
        !d_counts)
        return MGS_EINVAL;
    if (B > 0 && (!d_x || !d_batch)) return MGS_EINVAL;
    const KmLayout L = km_layout(B, D, K);
    if (!d_ws || ws_bytes < L.total) return MGS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    KmArgs a;
    std::memset(&a, 0, sizeof(a));
    a.x = d_x;
    a.batch = d_batch;
    a.xb = (float*)(ws + L.xb);
    a.assign = d_assign ? d_assign : (int32_t*)(ws + L.assign);
    a.keys = (uint32_t*)(ws + L.keys);
    a.keys_s = (uint32_t*)(ws + L.keys_s);
    a.pos = (int32_t*)(ws + L.pos);
    a.pos_s = (int32_t*)(ws + L.pos_s);
    a.cb = d_cb;
    a.counts = d_counts;
    a.status = (mgs_status_block*)ws;
    a.N = N;
    a.B = B;
    a.D = D;
    a.K = K;
    int rc = mgs_fill<uint32_t>((uint32_t*)ws, 64, 0u, s);
    if (rc) return rc;
    if (B == 0) return MGS_OK;
    hipLaunchKernelGGL(km_gather_kernel, dim3(km_blocks(B * D)), dim3(256), 0, s, a);
    rc = mgs_last_launch();
    if (rc) return rc;
    // nearest centers of the batch rows; its status word (non-finite rows or
    // centers) is folded into this call's below
    char* vq_ws = ws + L.vq;
    rc = mgs_vq_assign(a.xb, B, D, d_cb, K, a.assign, nullptr, nullptr, vq_ws,
                       mgs_vq_assign_ws_bytes(B, D, K), stream);
    if (rc) return rc;
    hipLaunchKernelGGL(km_status_kernel, dim3(1), dim3(64), 0, s, (const mgs_status_block*)vq_ws, a.status);
    // the batch positions grouped by center, batch order kept within a center
    hipLaunchKernelGGL(km_keys_kernel, dim3(km_blocks(B)), dim3(256), 0, s, a);
    rc = mgs_last_launch();
    if (rc) return rc;
    size_t sort_bytes = L.sort_bytes;
    if (rocprim::radix_sort_pairs((void*)(ws + L.sort), sort_bytes, (const uint32_t*)a.keys, a.keys_s,
                                  (const int32_t*)a.pos, a.pos_s, (unsigned)B, 0, km_key_bits(K), s) !=
        hipSuccess)
        return MGS_EDEVICE;
    // one wave per center (grid-stride over the centers)
    const int64_t waves = std::min<int64_t>(K, 1 << 16);
    hipLaunchKernelGGL(km_center_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
    return mgs_last_launch();
}

// ------------------------------------------------------------------ retention
// Paper, same paragraph: the budget left after the essential components keeps
// the original SH vectors of the most important Gaussians; they are appended
// to the codebook and coded with it.  Here: the r retained rows (ascending
// Gaussian index, the selection of mgs_prune_select with one count r) are
// copied after the K codewords and their index entries point at them.
namespace mgs {
namespace {

__global__ void vq_retain_kernel(const float* __restrict__ x, int64_t N, int D,
                                 const int32_t* __restrict__ top, int64_t r, float* cb_ext, int K,
                                 int32_t* idx, mgs_status_block* status) {
    const int64_t total = r * D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / D;
        const int d = (int)(i - e * D);
        const int64_t g = top[e];
        if (g < 0 || g >= N) {
            if (d == 0 && status) atomicOr(&status->nonfinite, 2u);
            continue;
        }
        cb_ext[((int64_t)K + e) * D + d] = x[g * D + d];
        if (d == 0) idx[g] = (int32_t)(K + e);
    }
}

}  // namespace
}  // namespace mgs

extern "C" int64_t mgs_vq_retain_count(int64_t remaining_bits, int64_t N, int32_t D) {
    if (remaining_bits <= 0 || N <= 0 || D < 1) return 0;
    return std::min<int64_t>(N, remaining_bits / (32 * (int64_t)D));
}

extern "C" int mgs_vq_retain(const float* d_x, int64_t N, int32_t D, const int32_t* d_top, int64_t r,
                             float* d_cb_ext, int32_t K, int32_t* d_idx, void* d_ws, size_t ws_bytes,
                             void* stream) {
    using namespace mgs;
    if (N < 0 || D < 1 || D > MGS_MAX_VQ_DIM || K < 0 || r < 0 || r > N || (int64_t)K + r >= ((int64_t)1 << 31))
        return MGS_EINVAL;
    if (r > 0 && (!d_x || !d_top || !d_cb_ext || !d_idx)) return MGS_EINVAL;
    if (!d_ws || ws_bytes < MGS_STATUS_BYTES) return MGS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    auto* status = (mgs_status_block*)d_ws;
    int rc = mgs_fill<uint32_t>((uint32_t*)d_ws, 64, 0u, s);
    if (rc || r == 0) return rc;
    hipLaunchKernelGGL(vq_retain_kernel, dim3(km_blocks(r * D)), dim3(256), 0, s, d_x, N, (int)D, d_top, r,
                       d_cb_ext, (int)K, d_idx, status);
    return mgs_last_launch();
}
