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
// A merged node keeps the slot of its first leaf.  Output per channel:
// coefficient 0 = DC (the root's value), then the AC coefficients in the
// order they are made (step by step, within a step in Morton order).  FP64
// arithmetic in exactly the order above, FP32 storage.  The inverse undoes
// the merges in reverse:  a1 = (sqrt(w1) L - sqrt(w2) H) / sqrt(w1 + w2),
//                         a2 = (sqrt(w2) L + sqrt(w1) H) / sqrt(w1 + w2).
//
// The merge structure follows from the codes alone, without running the
// steps: every merge joins the leaves on the two sides of one boundary i
// between neighbouring codes (N - 1 boundaries, N - 1 merges).  With d the
// highest bit in which code[i] and code[i + 1] differ, the merge happens at
// step d and joins the leaves [L, i] and [i + 1, R], the run of codes that
// agree with code[i] above bit d (every boundary inside either side differs
// lower, so each side is one node by then): L and R are binary searches in
// the sorted codes, the weights are i - L + 1 and R - i, the slots L and
// i + 1.  The AC index of the merge is its rank in (step, boundary) order:
// per-block counts of each step, a scan over (step, block), and a scatter
// that ranks a block's boundaries of each step with wavefront ballots.  The
// values then go through one launch per step over that step's merges only;
// they are stored node-major ([N][C]) and a merge is done by a team of lanes,
// one per channel, so its two nodes' rows are read and written whole however
// far apart the nodes are (with one node per lane and channel-major values a
// merge touched a separate cache line per channel and node).
#include <cstring>

#include "common.h"

namespace mgs {
namespace {

constexpr int RH_THREADS = 256;
constexpr int RH_ITEMS = 8;                          // boundaries per thread
constexpr int RH_SPAN = RH_THREADS * RH_ITEMS;       // per block
constexpr int RH_MAX_BLOCKS = 4096;                  // N - 1 <= RH_SPAN * RH_MAX_BLOCKS
constexpr int RH_BINS = 64;                          // merge steps (3 depth <= 63)
constexpr int RH_TEAM = 32;                          // lanes per merge (one channel each)
constexpr int RH_TEAMS = RH_THREADS / RH_TEAM;
constexpr int RH_GROUP = 16;                         // consecutive merges per block iteration

struct RahtArgs {
    const uint64_t* codes;
    int64_t N;
    int32_t C;
    int32_t depth;
    int64_t ld;
    const float* attr;     // forward input [C][ld]
    const float* coef_in;  // inverse input [C][ld]
    float* coef;           // forward output [C][ld]
    float* attr_out;       // inverse output [C][ld]
    double* val;           // [N][C] node values by slot (a node's channels adjacent)
    uint8_t* dstep;        // [N - 1] merge step of each boundary
    int32_t* lb;           // [N - 1] first leaf of each boundary's merge
    int32_t* rb;           // [N - 1] last leaf
    int64_t* cnt;          // [RH_BINS][nblk] boundaries per (step, block), then their first AC index
    int64_t* tot;          // [RH_BINS] boundaries per step
    int64_t* ac_base;      // [RH_BINS + 1] first AC index of each step
    int32_t* pa;           // [N - 1] per AC index: slot of the first node
    int32_t* pb;           //                       slot of the second node
    int64_t* wa;           //                       weights
    int64_t* wb;
    mgs_status_block* status;
    int32_t nblk;          // blocks over the N - 1 boundaries
    int32_t values;        // forward: the leaves' values are loaded
};

// The codes must increase and stay below 2^(3 depth).
__global__ void raht_init_kernel(RahtArgs a) {
    const int64_t lim = a.depth >= 21 ? 0 : ((int64_t)1 << (3 * a.depth));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = a.codes[i];
        if ((i > 0 && a.codes[i - 1] >= c) || (lim && c >= (uint64_t)lim)) atomicOr(&a.status->nonfinite, 4u);
    }
    if (blockIdx.x == 0)
        for (int b = threadIdx.x; b < RH_BINS; b += blockDim.x) a.tot[b] = 0;
}

// Transposes between the [C][ld] FP32 attribute layout and the [N][C] FP64
// node values through an LDS tile of 64 nodes x 32 channels, so that both
// sides are read and written in runs.
constexpr int RH_TILE_N = 64, RH_TILE_C = 32;

__global__ __launch_bounds__(RH_THREADS) void raht_load_kernel(RahtArgs a) {
    __shared__ double t[RH_TILE_C][RH_TILE_N + 1];
    for (int64_t i0 = (int64_t)blockIdx.x * RH_TILE_N; i0 < a.N; i0 += (int64_t)gridDim.x * RH_TILE_N) {
        const int nn = (int)std::min<int64_t>(RH_TILE_N, a.N - i0);
        for (int k0 = 0; k0 < a.C; k0 += RH_TILE_C) {
            const int nk = std::min(RH_TILE_C, a.C - k0);
            for (int e = threadIdx.x; e < nk * RH_TILE_N; e += RH_THREADS) {
                const int kk = e / RH_TILE_N, n = e % RH_TILE_N;
                if (n < nn) t[kk][n] = (double)a.attr[(int64_t)(k0 + kk) * a.ld + i0 + n];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < nk * nn; e += RH_THREADS) {
                const int n = e / nk, kk = e % nk;
                a.val[(i0 + n) * a.C + k0 + kk] = t[kk][n];
            }
            __syncthreads();
        }
    }
}

// The merge across boundary i: its step d and the leaf range [L, R] it joins
// ([L, i] first node, [i + 1, R] second).  Codes that do not increase give a
// harmless stand-in (d = 0, L = i, R = i + 1; the status flag is raised by
// the init kernel) so every index stays in bounds.
struct Boundary {
    int d;
    int64_t L, R;
};

__device__ __forceinline__ int boundary_step(const RahtArgs& a, int64_t i) {
    const uint64_t c0 = a.codes[i], c1 = a.codes[i + 1];
    if (c1 <= c0) return 0;
    const int d = 63 - __clzll((long long)(c0 ^ c1));
    return d >= 3 * a.depth ? RH_BINS - 1 : d;  // beyond the grid: never merged (flagged by init)
}

__device__ __forceinline__ Boundary boundary(const RahtArgs& a, int64_t i) {
    const uint64_t c0 = a.codes[i], c1 = a.codes[i + 1];
    Boundary b{0, i, i + 1};
    if (c1 <= c0) return b;
    const int d = 63 - __clzll((long long)(c0 ^ c1));
    if (d >= 3 * a.depth) {
        b.d = RH_BINS - 1;
        return b;
    }
    b.d = d;
    const int sh = d + 1;                              // <= 63
    const uint64_t lo_code = (c0 >> sh) << sh;         // first code of the run
    const uint64_t hi_code = lo_code + (1ull << sh);   // first code past it
    // a run spans at most 2^sh codes, hence at most that many leaves
    const int64_t span = sh >= 62 ? a.N : std::min<int64_t>(a.N, (int64_t)1 << sh);
    // L: first j in [max(0, i + 1 - span), i] with code[j] >= lo_code
    int64_t lo = std::max<int64_t>(0, i + 1 - span), hi = i;
    while (lo < hi) {
        const int64_t m = lo + ((hi - lo) >> 1);
        if (a.codes[m] >= lo_code) hi = m;
        else lo = m + 1;
    }
    b.L = lo;
    // R: last j in [i + 1, min(N - 1, i + span)] with code[j] < hi_code
    lo = i + 1;
    hi = std::min<int64_t>(a.N - 1, i + span);
    while (lo < hi) {
        const int64_t m = lo + ((hi - lo + 1) >> 1);
        if (a.codes[m] < hi_code) lo = m;
        else hi = m - 1;
    }
    b.R = lo;
    return b;
}

// Boundaries of each step in this block (boundary i = blockIdx.x * RH_SPAN +
// e * RH_THREADS + threadIdx.x).
__global__ __launch_bounds__(RH_THREADS) void raht_count_kernel(RahtArgs a) {
    __shared__ uint32_t h[RH_BINS];
    for (int b = threadIdx.x; b < RH_BINS; b += RH_THREADS) h[b] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * RH_SPAN + threadIdx.x;
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        if (i >= a.N - 1) break;
        const int d = boundary_step(a, i);
        a.dstep[i] = (uint8_t)d;
        atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < RH_BINS; b += RH_THREADS) {
        a.cnt[(int64_t)b * a.nblk + blockIdx.x] = h[b];
        if (h[b]) atomicAdd((unsigned long long*)&a.tot[b], (unsigned long long)h[b]);
    }
}

// The leaf range of every boundary's merge (one boundary per thread: the
// binary searches of many boundaries are in flight at once).
__global__ void raht_bounds_kernel(RahtArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N - 1;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Boundary b = boundary(a, i);
        a.lb[i] = (int32_t)b.L;
        a.rb[i] = (int32_t)b.R;
    }
}

// One block per step: the first AC index of each (step, block) -- the steps
// before this one, then this step's counts of the earlier blocks -- in place,
// and the first AC index of the step.
__global__ __launch_bounds__(RH_THREADS) void raht_scan_kernel(RahtArgs a) {
    __shared__ int64_t v[RH_MAX_BLOCKS];
    __shared__ int64_t part[RH_THREADS];
    const int st = blockIdx.x;
    int64_t base = 0;
    for (int b = 0; b < st; ++b) base += a.tot[b];
    int64_t* c = a.cnt + (int64_t)st * a.nblk;
    for (int j = threadIdx.x; j < a.nblk; j += RH_THREADS) v[j] = c[j];
    __syncthreads();
    constexpr int PER = RH_MAX_BLOCKS / RH_THREADS;
    const int j0 = threadIdx.x * PER;
    int64_t sum = 0;
    for (int e = 0; e < PER; ++e)
        if (j0 + e < a.nblk) sum += v[j0 + e];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < RH_THREADS; o <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = base + part[threadIdx.x] - sum;
    for (int e = 0; e < PER; ++e)
        if (j0 + e < a.nblk) {
            const int64_t x = v[j0 + e];
            v[j0 + e] = run;
            run += x;
        }
    __syncthreads();
    for (int j = threadIdx.x; j < a.nblk; j += RH_THREADS) c[j] = v[j];
    if (threadIdx.x == 0) {
        a.ac_base[st] = base;
        if (st == RH_BINS - 1) a.ac_base[RH_BINS] = base + a.tot[st];
    }
}

// Every boundary's merge at its AC index: the block's offset for the step,
// plus the boundaries of that step in earlier (round, wave) pairs of the
// block, plus the lanes below with the same step (lanes grouped by step with
// six ballots, one per bit of the step).
__global__ __launch_bounds__(RH_THREADS) void raht_pairs_kernel(RahtArgs a) {
    constexpr int NW = RH_THREADS / MGS_WAVE;
    __shared__ uint32_t cw[RH_ITEMS][NW][RH_BINS];
    for (int j = threadIdx.x; j < RH_ITEMS * NW * RH_BINS; j += RH_THREADS) (&cw[0][0][0])[j] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & (MGS_WAVE - 1), wave = threadIdx.x / MGS_WAVE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t i0 = (int64_t)blockIdx.x * RH_SPAN + threadIdx.x;
    int bin[RH_ITEMS];
    uint32_t rank[RH_ITEMS];
#pragma unroll
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        const bool valid = i < a.N - 1;
        const int b = valid ? (int)a.dstep[i] : 0;
        bin[e] = b;
        uint64_t eq = __ballot(valid);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const uint64_t m = __ballot(valid && ((b >> k) & 1));
            eq &= ((b >> k) & 1) ? m : ~m;
        }
        rank[e] = (uint32_t)__popcll(eq & lt);
        if (valid && (eq & lt) == 0ull) cw[e][wave][b] = (uint32_t)__popcll(eq);
    }
    __syncthreads();
    if (threadIdx.x < RH_BINS) {
        uint32_t run = 0;
        for (int e = 0; e < RH_ITEMS; ++e)
            for (int w = 0; w < NW; ++w) {
                const uint32_t v = cw[e][w][threadIdx.x];
                cw[e][w][threadIdx.x] = run;
                run += v;
            }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < RH_ITEMS; ++e) {
        const int64_t i = i0 + (int64_t)e * RH_THREADS;
        if (i >= a.N - 1) continue;
        const int b = bin[e];
        const int64_t p = a.cnt[(int64_t)b * a.nblk + blockIdx.x] + cw[e][wave][b] + rank[e];
        const int64_t L = a.lb[i], R = a.rb[i];
        a.pa[p] = (int32_t)L;
        a.pb[p] = (int32_t)(i + 1);
        a.wa[p] = i - L + 1;
        a.wb[p] = R - i;
    }
}

// The merges of step s (independent of each other), RH_GROUP consecutive AC
// indices per block iteration: a team of RH_TEAM lanes takes one merge, lane
// k channel k (channels beyond the team in further rounds), so the two
// nodes' rows are read and written whole; the coefficients of the group go
// through LDS and out as runs of consecutive AC indices per channel.
__global__ __launch_bounds__(RH_THREADS) void raht_merge_kernel(RahtArgs a, int s) {
    __shared__ float hs[RH_TEAM][RH_GROUP];
    const int64_t b0 = a.ac_base[s], b1 = a.ac_base[s + 1];
    const int team = threadIdx.x / RH_TEAM, tl = threadIdx.x % RH_TEAM;
    for (int64_t g0 = b0 + (int64_t)blockIdx.x * RH_GROUP; g0 < b1; g0 += (int64_t)gridDim.x * RH_GROUP) {
        const int ng = (int)std::min<int64_t>(RH_GROUP, b1 - g0);
        for (int k0 = 0; k0 < a.C; k0 += RH_TEAM) {
            const int k = k0 + tl;
            for (int q = team; q < ng; q += RH_TEAMS) {
                const int64_t p = g0 + q;
                const int32_t sa = a.pa[p], sb = a.pb[p];
                const int64_t w1 = a.wa[p], w2 = a.wb[p];
                if (k < a.C) {
                    const double s1 = sqrt((double)w1), s2 = sqrt((double)w2), sw = sqrt((double)(w1 + w2));
                    double* va = a.val + (int64_t)sa * a.C;
                    const double a1 = va[k], a2 = a.val[(int64_t)sb * a.C + k];
                    const double L = (s1 * a1 + s2 * a2) / sw;
                    const double H = (s1 * a2 - s2 * a1) / sw;
                    va[k] = L;
                    hs[tl][q] = (float)H;
                }
            }
            __syncthreads();
            const int nk = std::min(RH_TEAM, a.C - k0);
            for (int j = threadIdx.x; j < nk * RH_GROUP; j += RH_THREADS) {
                const int kk = j / RH_GROUP, q = j % RH_GROUP;
                if (q < ng) a.coef[(int64_t)(k0 + kk) * a.ld + 1 + g0 + q] = hs[kk][q];
            }
            __syncthreads();
        }
    }
}

// DC coefficients: the value of the root (slot of the first leaf).
__global__ void raht_dc_kernel(RahtArgs a) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.C; k += gridDim.x * blockDim.x)
        a.coef[(int64_t)k * a.ld] = (float)a.val[k];  // slot 0, channel k
}

// Inverse: the root's value from the DC, then the merges of one step undone
// (steps in reverse order; the merges of a step are independent).
__global__ void raht_inv_init_kernel(RahtArgs a) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < a.C; k += gridDim.x * blockDim.x)
        a.val[k] = (double)a.coef_in[(int64_t)k * a.ld];
}

// The inverse of one step in the same layout: the group's coefficients come
// in through LDS as runs per channel, a team undoes one merge.
__global__ __launch_bounds__(RH_THREADS) void raht_unmerge_kernel(RahtArgs a, int s) {
    __shared__ float hs[RH_TEAM][RH_GROUP];
    const int64_t b0 = a.ac_base[s], b1 = a.ac_base[s + 1];
    const int team = threadIdx.x / RH_TEAM, tl = threadIdx.x % RH_TEAM;
    for (int64_t g0 = b0 + (int64_t)blockIdx.x * RH_GROUP; g0 < b1; g0 += (int64_t)gridDim.x * RH_GROUP) {
        const int ng = (int)std::min<int64_t>(RH_GROUP, b1 - g0);
        for (int k0 = 0; k0 < a.C; k0 += RH_TEAM) {
            const int nk = std::min(RH_TEAM, a.C - k0);
            for (int j = threadIdx.x; j < nk * RH_GROUP; j += RH_THREADS) {
                const int kk = j / RH_GROUP, q = j % RH_GROUP;
                if (q < ng) hs[kk][q] = a.coef_in[(int64_t)(k0 + kk) * a.ld + 1 + g0 + q];
            }
            __syncthreads();
            const int k = k0 + tl;
            for (int q = team; q < ng; q += RH_TEAMS) {
                const int64_t p = g0 + q;
                const int32_t sa = a.pa[p], sb = a.pb[p];
                const int64_t w1 = a.wa[p], w2 = a.wb[p];
                if (k < a.C) {
                    const double s1 = sqrt((double)w1), s2 = sqrt((double)w2), sw = sqrt((double)(w1 + w2));
                    double* va = a.val + (int64_t)sa * a.C;
                    const double L = va[k];
                    const double H = (double)hs[tl][q];
                    va[k] = (s1 * L - s2 * H) / sw;
                    a.val[(int64_t)sb * a.C + k] = (s2 * L + s1 * H) / sw;
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(RH_THREADS) void raht_store_kernel(RahtArgs a) {
    __shared__ double t[RH_TILE_C][RH_TILE_N + 1];
    for (int64_t i0 = (int64_t)blockIdx.x * RH_TILE_N; i0 < a.N; i0 += (int64_t)gridDim.x * RH_TILE_N) {
        const int nn = (int)std::min<int64_t>(RH_TILE_N, a.N - i0);
        for (int k0 = 0; k0 < a.C; k0 += RH_TILE_C) {
            const int nk = std::min(RH_TILE_C, a.C - k0);
            for (int e = threadIdx.x; e < nk * nn; e += RH_THREADS) {
                const int n = e / nk, kk = e % nk;
                t[kk][n] = a.val[(i0 + n) * a.C + k0 + kk];
            }
            __syncthreads();
            for (int e = threadIdx.x; e < nk * RH_TILE_N; e += RH_THREADS) {
                const int kk = e / RH_TILE_N, n = e % RH_TILE_N;
                if (n < nn) a.attr_out[(int64_t)(k0 + kk) * a.ld + i0 + n] = (float)t[kk][n];
            }
            __syncthreads();
        }
    }
}

struct RahtLayout {
    size_t val, dstep, lb, rb, cnt, tot, ac, pa, pb, wa, wb, total;
    int nblk, steps;
};

RahtLayout raht_layout(int64_t N, int32_t C, int32_t depth) {
    RahtLayout L;
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    L.nblk = (int)((N - 1 + RH_SPAN - 1) / RH_SPAN);
    L.steps = 3 * depth;
    size_t o = MGS_STATUS_BYTES;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += mgs_align_up(bytes, 256);
        return at;
    };
    L.val = take(sizeof(double) * n * (size_t)C);
    L.dstep = take(n);
    L.lb = take(sizeof(int32_t) * n);
    L.rb = take(sizeof(int32_t) * n);
    L.cnt = take(sizeof(int64_t) * (size_t)RH_BINS * (size_t)std::max(L.nblk, 1));
    L.tot = take(sizeof(int64_t) * RH_BINS);
    L.ac = take(sizeof(int64_t) * (RH_BINS + 1));
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

// Leaf values (forward) and the merge structure: every merge's step, slots
// and weights at its AC index.
int raht_structure(RahtArgs& a, const RahtLayout& L, hipStream_t s) {
    hipLaunchKernelGGL(raht_init_kernel, dim3(rh_grid(a.N)), dim3(256), 0, s, a);
    if (a.values) hipLaunchKernelGGL(raht_load_kernel, dim3(rh_grid(a.N / 4 + 1)), dim3(RH_THREADS), 0, s, a);
    if (L.nblk > 0) {
        hipLaunchKernelGGL(raht_count_kernel, dim3(L.nblk), dim3(RH_THREADS), 0, s, a);
        hipLaunchKernelGGL(raht_bounds_kernel, dim3(rh_grid(a.N - 1)), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(raht_scan_kernel, dim3(RH_BINS), dim3(RH_THREADS), 0, s, a);
    if (L.nblk > 0) hipLaunchKernelGGL(raht_pairs_kernel, dim3(L.nblk), dim3(RH_THREADS), 0, s, a);
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
    a.depth = depth;
    a.ld = ld;
    a.val = (double*)(ws + L.val);
    a.dstep = (uint8_t*)(ws + L.dstep);
    a.lb = (int32_t*)(ws + L.lb);
    a.rb = (int32_t*)(ws + L.rb);
    a.cnt = (int64_t*)(ws + L.cnt);
    a.tot = (int64_t*)(ws + L.tot);
    a.ac_base = (int64_t*)(ws + L.ac);
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
    if (!rc) rc = raht_structure(a, L, s);
    if (rc) return rc;
    for (int st = 0; st < L.steps; ++st)
        hipLaunchKernelGGL(raht_merge_kernel, dim3(rh_grid(N / 2 + 1)), dim3(RH_THREADS), 0, s, a, st);
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
    if (!rc) rc = raht_structure(a, L, s);
    if (rc) return rc;
    hipLaunchKernelGGL(raht_inv_init_kernel, dim3(1), dim3(64), 0, s, a);
    for (int st = L.steps - 1; st >= 0; --st)
        hipLaunchKernelGGL(raht_unmerge_kernel, dim3(rh_grid(N / 2 + 1)), dim3(RH_THREADS), 0, s, a, st);
    hipLaunchKernelGGL(raht_store_kernel, dim3(rh_grid(N / 4 + 1)), dim3(RH_THREADS), 0, s, a);
    return mgs_last_launch();
}
