// Region-Adaptive Hierarchical Transform of the attributes over the
// voxelized positions.  Paper: section "Attribute Transformation",
// paragraph "Region Adaptive Hierarchical Transform" (transform T_1, its 2-D
// example, leaf weight 1, merged weight the sum of the child weights,
// unmatched coefficients passing to the next layer, one DC and N - 1 AC
// coefficients per channel).
//
// Positions are Morton codes (per level: x in bit 0, y in bit 1, z in bit 2),
// strictly increasing.  Step s = 0, 1, ..., 3 * depth - 1 merges, along the
// axis of bit s, every two live nodes whose codes agree above bit s: the one
// with bit s clear (weight w1, value a1) and the one with it set (w2, a2):
//   L = (sqrt(w1) a1 + sqrt(w2) a2) / sqrt(w1 + w2)      (goes up, weight w1 + w2)
//   H = (sqrt(w1) a2 - sqrt(w2) a1) / sqrt(w1 + w2)      (AC coefficient)
// A merged node keeps the slot of its first node, so live nodes stay in
// Morton order.  Output per channel: coefficient 0 = DC (the root's value),
// then the AC coefficients in the order they are made (step by step, within
// a step in Morton order).  FP64 arithmetic in exactly the order above, FP32
// storage.  The inverse recomputes the merges from the positions and undoes
// them in reverse:  a1 = (sqrt(w1) L - sqrt(w2) H) / sqrt(w1 + w2),
//                   a2 = (sqrt(w2) L + sqrt(w1) H) / sqrt(w1 + w2).
//
// Each step is three launches over the live-node list: pair flags and block
// sums, a one-block scan of the block sums (which also advances the live and
// AC counts kept on the device), and the merges with the compaction of the
// list.  Nothing is read back to the host between steps.  Consecutive lanes
// take consecutive live nodes, so the list, the codes and (while the live
// slots are dense) the values are read coalesced.
#include <cstring>

#include "common.h"

namespace mgs {
namespace {

constexpr int RH_THREADS = 256;
constexpr int RH_ITEMS = 8;                          // live nodes per thread
constexpr int RH_SPAN = RH_THREADS * RH_ITEMS;       // per block
constexpr int RH_MAX_BLOCKS = RH_THREADS * 16;       // one-block scan capacity

struct RahtArgs {
    const uint64_t* codes;
    int64_t N;
    int32_t C;
    int64_t ld;
    const float* attr;     // forward input [C][ld]
    const float* coef_in;  // inverse input [C][ld]
    float* coef;           // forward output [C][ld]
    float* attr_out;       // inverse output [C][ld]
    double* val;           // [C][N] node values by slot
    int64_t* w;            // [N] node weights by slot
    int32_t* live[2];      // live slot lists (ping-pong)
    int64_t* bsum;         // [nblk] packed block sums: pairs | kept << 32
    int64_t* n_live;       // [steps + 1]
    int64_t* ac_base;      // [steps + 1]
    int32_t* pa;           // [N] per AC index: first slot of the pair
    int32_t* pb;           //                   second slot
    int64_t* wa;           //                   weights
    int64_t* wb;
    mgs_status_block* status;
    int32_t nblk;
    int32_t values;        // forward pass also carries the values
};

// Slot list, weights and values of the leaves; the codes must increase.
__global__ void raht_init_kernel(RahtArgs a, int depth) {
    const int64_t lim = depth >= 21 ? 0 : ((int64_t)1 << (3 * depth));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        a.live[0][i] = (int32_t)i;
        a.w[i] = 1;
        const uint64_t c = a.codes[i];
        if ((i > 0 && a.codes[i - 1] >= c) || (lim && c >= (uint64_t)lim)) atomicOr(&a.status->nonfinite, 4u);
        if (a.values)
            for (int k = 0; k < a.C; ++k) a.val[(int64_t)k * a.N + i] = (double)a.attr[(int64_t)k * a.ld + i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.n_live[0] = a.N;
        a.ac_base[0] = 0;
    }
}

// Live node i at step s: first of a pair (bit s clear, the next live node
// has the same parent) or second of one.
struct PairFlags {
    bool first, second;
};

__device__ __forceinline__ PairFlags pair_flags(const RahtArgs& a, const int32_t* live, int64_t n, int64_t i,
                                                int s) {
    const uint64_t key = a.codes[live[i]] >> s;
    PairFlags f{false, false};
    if ((key & 1u) == 0) {
        f.first = i + 1 < n && (a.codes[live[i + 1]] >> s) >> 1 == key >> 1;
    } else {
        f.second = i > 0 && (a.codes[live[i - 1]] >> s) >> 1 == key >> 1;
    }
    return f;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v) {
    __shared__ int64_t part[RH_THREADS / MGS_WAVE];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, MGS_WAVE);
    if ((threadIdx.x & (MGS_WAVE - 1)) == 0) part[threadIdx.x / MGS_WAVE] = v;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int k = 0; k < RH_THREADS / MGS_WAVE; ++k) t += part[k];
    __syncthreads();
    return t;
}

// Exclusive scan of one value per thread over the block; also the total.
__device__ __forceinline__ int64_t block_exscan_i64(int64_t v, int64_t& total) {
    __shared__ int64_t sc[RH_THREADS];
    sc[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < RH_THREADS; o <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)o ? sc[threadIdx.x - o] : 0;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    total = sc[RH_THREADS - 1];
    const int64_t ex = sc[threadIdx.x] - v;
    __syncthreads();
    return ex;
}

__global__ __launch_bounds__(RH_THREADS) void raht_count_kernel(RahtArgs a, int s) {
    const int32_t* live = a.live[s & 1];
    const int64_t n = a.n_live[s];
    int64_t v = 0;
    const int64_t i0 = (int64_t)blockIdx.x * RH_SPAN + threadIdx.x;
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        if (i >= n) break;
        const PairFlags f = pair_flags(a, live, n, i, s);
        v += (int64_t)f.first + ((int64_t)(!f.second) << 32);
    }
    v = block_sum_i64(v);
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = v;
}

// One block: exclusive scan of the block sums in place; the next live count
// and the AC base of the next step.
__global__ __launch_bounds__(RH_THREADS) void raht_scan_kernel(RahtArgs a, int s) {
    constexpr int PER = RH_MAX_BLOCKS / RH_THREADS;
    int64_t loc[PER];
    int64_t t = 0;
    for (int e = 0; e < PER; ++e) {
        const int b = threadIdx.x * PER + e;
        loc[e] = b < a.nblk ? a.bsum[b] : 0;
        t += loc[e];
    }
    int64_t total = 0;
    int64_t off = block_exscan_i64(t, total);
    for (int e = 0; e < PER; ++e) {
        const int b = threadIdx.x * PER + e;
        if (b < a.nblk) a.bsum[b] = off;
        off += loc[e];
    }
    if (threadIdx.x == 0) {
        a.n_live[s + 1] = total >> 32;
        a.ac_base[s + 1] = a.ac_base[s] + (total & 0xFFFFFFFFll);
    }
}

// The block's live nodes are taken in rounds of RH_THREADS consecutive ones
// (consecutive lanes, consecutive nodes: coalesced reads of the list, the
// codes and the values); a node's output positions follow node order, from
// wavefront ballots: per (round, wave) counts, one wavefront's exclusive scan
// of them, plus the lanes below.
__global__ __launch_bounds__(RH_THREADS) void raht_merge_kernel(RahtArgs a, int s) {
    constexpr int NW = RH_THREADS / MGS_WAVE;
    static_assert(RH_ITEMS * NW <= MGS_WAVE, "one (round, wave) count per lane of the scanning wavefront");
    __shared__ int64_t off[RH_ITEMS * NW];
    const int32_t* live = a.live[s & 1];
    int32_t* next = a.live[(s + 1) & 1];
    const int64_t n = a.n_live[s];
    const int lane = threadIdx.x & (MGS_WAVE - 1), wave = threadIdx.x / MGS_WAVE;
    const int64_t i0 = (int64_t)blockIdx.x * RH_SPAN + threadIdx.x;
    uint64_t mf[RH_ITEMS], mk[RH_ITEMS];
#pragma unroll
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        const PairFlags f = i < n ? pair_flags(a, live, n, i, s) : PairFlags{false, true};
        mf[e] = __ballot(f.first);
        mk[e] = __ballot(!f.second);
    }
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < RH_ITEMS; ++e)
            off[e * NW + wave] = (int64_t)__popcll(mf[e]) + ((int64_t)__popcll(mk[e]) << 32);
    }
    __syncthreads();
    if (wave == 0) {
        const int64_t v = lane < RH_ITEMS * NW ? off[lane] : 0;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < MGS_WAVE; o <<= 1) {
            const int64_t y = __shfl_up(incl, o, MGS_WAVE);
            if (lane >= o) incl += y;
        }
        if (lane < RH_ITEMS * NW) off[lane] = a.bsum[blockIdx.x] + incl - v;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        if (i >= n) continue;
        const int64_t o = off[e * NW + wave];
        const int32_t sa = live[i];
        if ((mf[e] >> lane) & 1ull) {
            const int64_t pos_pair = a.ac_base[s] + (o & 0xFFFFFFFFll) + __popcll(mf[e] & lt);
            const int32_t sb = live[i + 1];
            const int64_t w1 = a.w[sa], w2 = a.w[sb];
            a.pa[pos_pair] = sa;
            a.pb[pos_pair] = sb;
            a.wa[pos_pair] = w1;
            a.wb[pos_pair] = w2;
            if (a.values) {
                const double s1 = sqrt((double)w1), s2 = sqrt((double)w2), sw = sqrt((double)(w1 + w2));
#pragma unroll 4
                for (int k = 0; k < a.C; ++k) {
                    const double a1 = a.val[(int64_t)k * a.N + sa], a2 = a.val[(int64_t)k * a.N + sb];
                    const double L = (s1 * a1 + s2 * a2) / sw;
                    const double H = (s1 * a2 - s2 * a1) / sw;
                    a.val[(int64_t)k * a.N + sa] = L;
                    a.coef[(int64_t)k * a.ld + 1 + pos_pair] = (float)H;
                }
            }
            a.w[sa] = w1 + w2;
        }
        if ((mk[e] >> lane) & 1ull) next[(o >> 32) + __popcll(mk[e] & lt)] = sa;
    }
}

// DC coefficients: the value of the root (slot of the first leaf).
__global__ void raht_dc_kernel(RahtArgs a) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.C; k += gridDim.x * blockDim.x)
        a.coef[(int64_t)k * a.ld] = (float)a.val[(int64_t)k * a.N];
}

// Inverse: the root's value from the DC, then the merges of one step undone
// (steps in reverse order; the merges of a step are independent).
__global__ void raht_inv_init_kernel(RahtArgs a) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.C; k += gridDim.x * blockDim.x)
        a.val[(int64_t)k * a.N] = (double)a.coef_in[(int64_t)k * a.ld];
}

__global__ void raht_unmerge_kernel(RahtArgs a, int s) {
    const int64_t b0 = a.ac_base[s], b1 = a.ac_base[s + 1];
    for (int64_t p = b0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < b1;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sa = a.pa[p], sb = a.pb[p];
        const int64_t w1 = a.wa[p], w2 = a.wb[p];
        const double s1 = sqrt((double)w1), s2 = sqrt((double)w2), sw = sqrt((double)(w1 + w2));
#pragma unroll 4
        for (int k = 0; k < a.C; ++k) {
            const double L = a.val[(int64_t)k * a.N + sa];
            const double H = (double)a.coef_in[(int64_t)k * a.ld + 1 + p];
            a.val[(int64_t)k * a.N + sa] = (s1 * L - s2 * H) / sw;
            a.val[(int64_t)k * a.N + sb] = (s2 * L + s1 * H) / sw;
        }
    }
}

__global__ void raht_store_kernel(RahtArgs a) {
    const int64_t total = (int64_t)a.C * a.N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / a.N, j = i - k * a.N;
        a.attr_out[k * a.ld + j] = (float)a.val[i];
    }
}

struct RahtLayout {
    size_t val, w, live0, live1, bsum, counts, pa, pb, wa, wb, total;
    int nblk, steps;
};

RahtLayout raht_layout(int64_t N, int32_t C, int32_t depth) {
    RahtLayout L;
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    L.nblk = (int)((N + RH_SPAN - 1) / RH_SPAN);
    L.steps = 3 * depth;
    size_t o = MGS_STATUS_BYTES;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += mgs_align_up(bytes, 256);
        return at;
    };
    L.val = take(sizeof(double) * n * (size_t)C);
    L.w = take(sizeof(int64_t) * n);
    L.live0 = take(sizeof(int32_t) * n);
    L.live1 = take(sizeof(int32_t) * n);
    L.bsum = take(sizeof(int64_t) * (size_t)std::max(L.nblk, 1));
    L.counts = take(sizeof(int64_t) * 2 * (size_t)(L.steps + 1));
    L.pa = take(sizeof(int32_t) * n);
    L.pb = take(sizeof(int32_t) * n);
    L.wa = take(sizeof(int64_t) * n);
    L.wb = take(sizeof(int64_t) * n);
    L.total = o;
    return L;
}

unsigned rh_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

// The merge steps; with values the forward transform, without them only the
// structure (for the inverse).
int raht_steps(RahtArgs& a, const RahtLayout& L, int depth, hipStream_t s) {
    hipLaunchKernelGGL(raht_init_kernel, dim3(rh_grid(a.N)), dim3(256), 0, s, a, depth);
    for (int st = 0; st < L.steps; ++st) {
        hipLaunchKernelGGL(raht_count_kernel, dim3(L.nblk), dim3(RH_THREADS), 0, s, a, st);
        hipLaunchKernelGGL(raht_scan_kernel, dim3(1), dim3(RH_THREADS), 0, s, a, st);
        hipLaunchKernelGGL(raht_merge_kernel, dim3(L.nblk), dim3(RH_THREADS), 0, s, a, st);
    }
    return mgs_last_launch();
}

int raht_setup(RahtArgs& a, RahtLayout& L, const uint64_t* codes, int64_t N, int32_t C, int64_t ld,
               int32_t depth, void* d_ws, size_t ws_bytes) {
    if (N < 1 || N >= ((int64_t)1 << 31) || C < 1 || ld < N || depth < 1 || depth > 21 || !codes)
        return MGS_EINVAL;
    L = raht_layout(N, C, depth);
    if (L.nblk > RH_MAX_BLOCKS) return MGS_EINVAL;
    if (!d_ws || ws_bytes < L.total) return MGS_EWORKSPACE;
    char* ws = (char*)d_ws;
    std::memset(&a, 0, sizeof(a));
    a.codes = codes;
    a.N = N;
    a.C = C;
    a.ld = ld;
    a.val = (double*)(ws + L.val);
    a.w = (int64_t*)(ws + L.w);
    a.live[0] = (int32_t*)(ws + L.live0);
    a.live[1] = (int32_t*)(ws + L.live1);
    a.bsum = (int64_t*)(ws + L.bsum);
    a.n_live = (int64_t*)(ws + L.counts);
    a.ac_base = a.n_live + (L.steps + 1);
    a.pa = (int32_t*)(ws + L.pa);
    a.pb = (int32_t*)(ws + L.pb);
    a.wa = (int64_t*)(ws + L.wa);
    a.wb = (int64_t*)(ws + L.wb);
    a.status = (mgs_status_block*)ws;
    a.nblk = L.nblk;
    return MGS_OK;
}

}  // namespace
}  // namespace mgs

extern "C" size_t mgs_raht_ws_bytes(int64_t N, int32_t C, int32_t depth) {
    if (N < 1 || C < 1 || depth < 1 || depth > 21) return 0;
    return mgs::raht_layout(N, C, depth).total;
}

extern "C" int mgs_raht_forward(const uint64_t* d_codes, int64_t N, int32_t C, int32_t depth, const float* d_attr,
                                int64_t ld, float* d_coef, void* d_ws, size_t ws_bytes, void* stream) {
    using namespace mgs;
    RahtArgs a;
    RahtLayout L;
    int rc = raht_setup(a, L, d_codes, N, C, ld, depth, d_ws, ws_bytes);
    if (rc) return rc;
    if (!d_attr || !d_coef) return MGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    a.attr = d_attr;
    a.coef = d_coef;
    a.values = 1;
    rc = mgs_fill<uint32_t>((uint32_t*)d_ws, 64, 0u, s);
    if (!rc) rc = raht_steps(a, L, depth, s);
    if (rc) return rc;
    hipLaunchKernelGGL(raht_dc_kernel, dim3(1), dim3(64), 0, s, a);
    return mgs_last_launch();
}

extern "C" int mgs_raht_inverse(const uint64_t* d_codes, int64_t N, int32_t C, int32_t depth, const float* d_coef,
                                int64_t ld, float* d_attr, void* d_ws, size_t ws_bytes, void* stream) {
    using namespace mgs;
    RahtArgs a;
    RahtLayout L;
    int rc = raht_setup(a, L, d_codes, N, C, ld, depth, d_ws, ws_bytes);
    if (rc) return rc;
    if (!d_attr || !d_coef) return MGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    a.coef_in = d_coef;
    a.attr_out = d_attr;
    a.values = 0;
    rc = mgs_fill<uint32_t>((uint32_t*)d_ws, 64, 0u, s);
    if (!rc) rc = raht_steps(a, L, depth, s);
    if (rc) return rc;
    hipLaunchKernelGGL(raht_inv_init_kernel, dim3(1), dim3(64), 0, s, a);
    for (int st = L.steps - 1; st >= 0; --st)
        hipLaunchKernelGGL(raht_unmerge_kernel, dim3(rh_grid(N / 2 + 1)), dim3(256), 0, s, a, st);
    hipLaunchKernelGGL(raht_store_kernel, dim3(rh_grid((int64_t)C * N)), dim3(256), 0, s, a);
    return mgs_last_launch();
}
