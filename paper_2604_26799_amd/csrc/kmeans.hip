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
// applied to the batch's rows in order) reaches the same mean; the batched
// form needs no order.  Sums are FP64 atomics into the workspace (their order
// varies, so the FP64 mean is reproducible to about B * 2^-53 relative), the
// result is rounded to FP32 once.
#include <cstring>

#include "common.h"

namespace mgs {
namespace {

struct KmArgs {
    const float* x;
    const int64_t* batch;
    float* xb;          // [B][D] gathered batch rows
    int32_t* assign;    // [B]
    double* sums;       // [K][D]
    int64_t* nb;        // [K] rows of this batch per center
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

// Per-center FP64 sums and counts of the batch rows.
__global__ void km_accumulate_kernel(KmArgs a) {
    const int64_t total = a.B * a.D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / a.D;
        const int d = (int)(i - r * a.D);
        const int j = a.assign[r];
        if ((unsigned)j >= (unsigned)a.K) continue;  // rows the assignment flagged non-finite
        atomicAdd(&a.sums[(int64_t)j * a.D + d], (double)a.xb[i]);
        if (d == 0) atomicAdd((unsigned long long*)&a.nb[j], 1ull);
    }
}

// The running-mean update of every center that received rows.
__global__ void km_update_kernel(KmArgs a) {
    const int64_t total = (int64_t)a.K * a.D;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i / a.D;
        const int64_t n = a.nb[j];
        if (n == 0) continue;
        const int64_t v = a.counts[j];
        const double c = (double)a.cb[i];
        a.cb[i] = (float)(((double)v * c + a.sums[i]) / (double)(v + n));
    }
}

// The assignment's status word (non-finite rows or centers) into this call's.
__global__ void km_status_kernel(const mgs_status_block* vq, mgs_status_block* own) {
    if (threadIdx.x == 0 && vq->nonfinite) atomicOr(&own->nonfinite, vq->nonfinite);
}

// The absorbed-sample counts, after every value of the center is updated.
__global__ void km_counts_kernel(KmArgs a) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.K;
         j += (int64_t)gridDim.x * blockDim.x)
        a.counts[j] += a.nb[j];
}

struct KmLayout {
    size_t xb, assign, sums, nb, vq, total;
};

KmLayout km_layout(int64_t B, int32_t D, int32_t K) {
    KmLayout L;
    size_t o = MGS_STATUS_BYTES;
    L.xb = o;
    o += mgs_align_up(sizeof(float) * (size_t)std::max<int64_t>(B, 1) * D, 256);
    L.assign = o;
    o += mgs_align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(B, 1), 256);
    L.sums = o;
    o += mgs_align_up(sizeof(double) * (size_t)K * D, 256);
    L.nb = o;
    o += mgs_align_up(sizeof(int64_t) * (size_t)K, 256);
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
    a.sums = (double*)(ws + L.sums);
    a.nb = (int64_t*)(ws + L.nb);
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
    rc = mgs_fill<double>(a.sums, (int64_t)K * D, 0.0, s);
    if (!rc) rc = mgs_fill<int64_t>(a.nb, K, (int64_t)0, s);
    if (rc) return rc;
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
    hipLaunchKernelGGL(km_accumulate_kernel, dim3(km_blocks(B * D)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(km_update_kernel, dim3(km_blocks((int64_t)K * D)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(km_counts_kernel, dim3(km_blocks(K)), dim3(256), 0, s, a);
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
