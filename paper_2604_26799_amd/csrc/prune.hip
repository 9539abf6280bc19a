// Reserve-ratio pruning: for each keep count k_t, the k_t most important
// Gaussians (equal importance: smaller index first), in ascending index order.
// Paper: section "Gaussians Pruning" (the reserve ratio tau keeps the most
// important tau*N Gaussians and cuts the rest).
//
// Every Gaussian gets a unique 64-bit key
//     ck(i) = (desc(imp[i]) << 32) | i
// where desc() maps floats to uint32 so that larger importance gives a
// smaller key (-0 and +0 map alike).  The kept set of count k is exactly
// {i : ck(i) <= thr}, thr being the k-th smallest key, so ties need no
// special treatment.  thr is found per k by a radix select over six digits
// (13/11/8 bits of the importance key, then 11/11/10 bits of the index):
// one histogram pass over the importance per digit, each followed by a tiny
// per-k kernel that picks the digit holding the k-th key.  Passes after the
// first only count keys that still match a k's prefix, found through an LDS
// table indexed by the top digit.  A k whose key is the last of its digit
// bucket is resolved there (every lower threshold bit set), and a pass with
// no unresolved k exits at once: without ties across the k-th key the index
// digits cost nothing.  A compaction then writes each kept set in index
// order: per-chunk counts, a per-k scan over chunks, and a write pass that
// ranks kept elements with wavefront ballots; a block of the counting and
// writing passes takes one chunk and a group of k, sized for ~2048 blocks.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace mgs {
namespace {

constexpr int PR_LEVELS = 6;
constexpr int PR_BINS = 8192;  // bins of the widest digit
constexpr int PR_HIST_THREADS = 256;
constexpr int PR_CHUNK_THREADS = 256;
constexpr int PR_CHUNK_ROUNDS = 16;
constexpr int PR_CHUNK = PR_CHUNK_THREADS * PR_CHUNK_ROUNDS;  // elements per compaction block
// a wide first digit, so that few keys share a k's prefix in the second pass
// (those are counted with global atomics)
constexpr int PR_SHIFT[PR_LEVELS] = {51, 40, 32, 21, 10, 0};
constexpr int PR_BITS[PR_LEVELS] = {13, 11, 8, 11, 11, 10};

struct PruneState {
    uint64_t prefix;  // key bits fixed so far (above the current digit)
    int64_t rem;      // rank (1-based) of the wanted key within that prefix; 0: resolved
};

struct PruneArgs {
    const float* imp;
    mgs_status_block* status;
    PruneState* state;   // [T]
    uint32_t* hist0;     // [PR_BINS]
    uint32_t* histA;     // [T][PR_BINS]
    uint32_t* histB;     // [T][PR_BINS]
    uint32_t* cnt;       // [T][nblk]
    int32_t* kept;
    int64_t n;
    int64_t nblk;
    int32_t T;
    int32_t pad;
    int64_t k[MGS_MAX_RATIOS];
    int64_t koff[MGS_MAX_RATIOS];
};

__device__ __forceinline__ uint32_t desc_key(float v) {
    uint32_t b = __float_as_uint(v);
    if (b == 0x80000000u) b = 0u;                             // -0 -> +0
    uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // ascending in v
    return ~asc;                                              // descending in v
}

__device__ __forceinline__ uint64_t comp_key(const float* imp, int64_t i) {
    return ((uint64_t)desc_key(imp[i]) << 32) | (uint64_t)i;
}

__device__ __forceinline__ uint32_t digit(uint64_t ck, int level) {
    return (uint32_t)(ck >> PR_SHIFT[level]) & ((1u << PR_BITS[level]) - 1u);
}

__device__ __forceinline__ uint32_t* level_hist(const PruneArgs& a, int level, int t) {
    if (level == 0) return a.hist0;
    return ((level & 1) ? a.histA : a.histB) + (int64_t)t * PR_BINS;
}

// Level 0: histogram of the top digit over all keys (LDS-privatised).
__global__ __launch_bounds__(PR_HIST_THREADS) void prune_hist0_kernel(PruneArgs a) {
    __shared__ uint32_t h[PR_BINS];
    for (int i = threadIdx.x; i < PR_BINS; i += PR_HIST_THREADS) h[i] = 0u;
    __syncthreads();
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * PR_HIST_THREADS + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * PR_HIST_THREADS) {
        float v = a.imp[i];
        bad |= (uint32_t)!finite_f32(v);
        atomicAdd(&h[desc_key(v) >> (32 - PR_BITS[0])], 1u);
    }
    if (bad) atomicOr(&a.status->nonfinite, 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < PR_BINS; i += PR_HIST_THREADS)
        if (h[i]) atomicAdd(&a.hist0[i], h[i]);
}

// Levels 1..5: histogram of digit `level` over the keys matching a k's prefix.
__global__ __launch_bounds__(PR_HIST_THREADS) void prune_hist_kernel(PruneArgs a, int level) {
    __shared__ int16_t first[PR_BINS];
    __shared__ int16_t next[MGS_MAX_RATIOS];
    __shared__ uint64_t pre[MGS_MAX_RATIOS];
    for (int i = threadIdx.x; i < PR_BINS; i += PR_HIST_THREADS) first[i] = -1;
    __syncthreads();
    __shared__ int active;
    const int hs = PR_SHIFT[level - 1];  // bits at and above this shift are fixed
    if (threadIdx.x < a.T && a.k[threadIdx.x] > 0) pre[threadIdx.x] = a.state[threadIdx.x].prefix >> hs;
    __syncthreads();
    // Build the per-top-digit lists serially (T <= 64 entries) of the k whose
    // key is not resolved yet.
    if (threadIdx.x == 0) {
        int na = 0;
        for (int t = a.T - 1; t >= 0; --t) {
            if (a.k[t] <= 0 || a.state[t].rem == 0) continue;
            uint32_t d0 = (uint32_t)(a.state[t].prefix >> PR_SHIFT[0]);
            next[t] = first[d0];
            first[d0] = (int16_t)t;
            ++na;
        }
        active = na;
    }
    __syncthreads();
    if (active == 0) return;  // every k resolved at an earlier digit (no tie across it)
    for (int64_t i = (int64_t)blockIdx.x * PR_HIST_THREADS + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * PR_HIST_THREADS) {
        uint64_t ck = comp_key(a.imp, i);
        int t = first[ck >> PR_SHIFT[0]];
        if (t < 0) continue;
        const uint64_t hi = ck >> hs;
        const uint32_t d = digit(ck, level);
        for (; t >= 0; t = next[t])
            if (pre[t] == hi) atomicAdd(&level_hist(a, level, t)[d], 1u);
    }
}

// One block per k: pick the digit that holds the rem-th key of the prefix
// bucket, extend the prefix, and clear this k's histogram of the next level.
__global__ __launch_bounds__(256) void prune_select_kernel(PruneArgs a, int level) {
    const int t = blockIdx.x;
    if (a.k[t] <= 0) return;
    if (level > 0 && a.state[t].rem == 0) return;  // resolved
    __shared__ uint32_t part[256];
    __shared__ int64_t found_base;
    __shared__ uint32_t found_digit, found_count;
    const uint32_t* h = level_hist(a, level, t);
    const int nbins = 1 << PR_BITS[level];
    const int per = PR_BINS / 256;  // 32 bins per thread (only the first nbins used)
    const int b0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (int j = 0; j < per; ++j)
        if (b0 + j < nbins) mine += h[b0 + j];
    part[threadIdx.x] = mine;
    __syncthreads();
    // inclusive scan (Hillis-Steele) over the 256 partial sums
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    PruneState st = level == 0 ? PruneState{0ull, a.k[t]} : a.state[t];
    const int64_t before = threadIdx.x ? part[threadIdx.x - 1] : 0;
    if (before < st.rem && st.rem <= (int64_t)part[threadIdx.x]) {
        int64_t cum = before;
        for (int j = 0; j < per; ++j) {
            uint32_t c = (b0 + j < nbins) ? h[b0 + j] : 0u;
            if (cum + c >= st.rem) {
                found_digit = (uint32_t)(b0 + j);
                found_base = cum;
                found_count = c;
                break;
            }
            cum += c;
        }
    }
    __syncthreads();
    if (level + 1 < PR_LEVELS) {
        uint32_t* hn = level_hist(a, level + 1, t);
        for (int i = threadIdx.x; i < PR_BINS; i += 256) hn[i] = 0u;
    }
    if (threadIdx.x == 0) {
        st.prefix |= (uint64_t)found_digit << PR_SHIFT[level];
        st.rem -= found_base;
        if (st.rem == (int64_t)found_count) {
            // the wanted key is the last of its bucket: the whole bucket is
            // kept, and no other key lies between, so the threshold can take
            // every lower bit set (with distinct importances this happens
            // once the importance digits are fixed, and the index digits
            // need no pass)
            st.prefix |= (PR_SHIFT[level] ? (1ull << PR_SHIFT[level]) - 1ull : 0ull);
            st.rem = 0;
        }
        a.state[t] = st;
    }
}

// Compaction, phase counts: kept keys of ratios [blockIdx.y * tb, + tb) in
// one chunk (the chunk's keys are read once for the tb ratios).
__global__ __launch_bounds__(PR_CHUNK_THREADS) void prune_count_kernel(PruneArgs a, int tb) {
    __shared__ uint32_t wsum[PR_CHUNK_THREADS / MGS_WAVE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * PR_CHUNK;
    uint64_t ck[PR_CHUNK_ROUNDS];
#pragma unroll
    for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) {
        int64_t i = base + r * PR_CHUNK_THREADS + threadIdx.x;
        ck[r] = i < a.n ? comp_key(a.imp, i) : ~0ull;
    }
    const int t1 = min(a.T, (int)(blockIdx.y + 1) * tb);
    for (int t = blockIdx.y * tb; t < t1; ++t) {
        if (a.k[t] <= 0) continue;  // uniform; its counts are never read
        const uint64_t th = a.state[t].prefix;
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) c += (uint32_t)__popcll(__ballot(ck[r] <= th));
        if (lane == 0) wsum[wave] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t sum = 0;
            for (int w = 0; w < PR_CHUNK_THREADS / MGS_WAVE; ++w) sum += wsum[w];
            a.cnt[(int64_t)t * a.nblk + blockIdx.x] = sum;
        }
        __syncthreads();
    }
}

// Compaction, phase scan: exclusive prefix of the block counts, one block per k.
__global__ __launch_bounds__(1024) void prune_scan_kernel(PruneArgs a) {
    const int t = blockIdx.x;
    __shared__ uint32_t carry;
    __shared__ uint32_t part[1024];
    uint32_t* c = a.cnt + (int64_t)t * a.nblk;
    if (threadIdx.x == 0) carry = 0u;
    __syncthreads();
    for (int64_t b0 = 0; b0 < a.nblk; b0 += 1024) {
        int64_t b = b0 + threadIdx.x;
        uint32_t v = b < a.nblk ? c[b] : 0u;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            uint32_t x = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
            __syncthreads();
            part[threadIdx.x] += x;
            __syncthreads();
        }
        if (b < a.nblk) c[b] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
}

// Compaction, phase write, one block per (chunk, group of tb ratios): each
// kept key's position is the chunk's offset, plus the kept keys of earlier
// (round, wave) pairs (an exclusive scan of the 64 ballot counts by one
// wavefront), plus the lanes below.
__global__ __launch_bounds__(PR_CHUNK_THREADS) void prune_write_kernel(PruneArgs a, int tb) {
    constexpr int NW = PR_CHUNK_THREADS / MGS_WAVE;
    static_assert(PR_CHUNK_ROUNDS * NW == MGS_WAVE, "one count per lane of the scanning wavefront");
    __shared__ uint32_t off[PR_CHUNK_ROUNDS * NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * PR_CHUNK;
    uint64_t ck[PR_CHUNK_ROUNDS];
#pragma unroll
    for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) {
        int64_t i = base + r * PR_CHUNK_THREADS + threadIdx.x;
        ck[r] = i < a.n ? comp_key(a.imp, i) : ~0ull;
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int t1 = min(a.T, (int)(blockIdx.y + 1) * tb);
    for (int t = blockIdx.y * tb; t < t1; ++t) {
        if (a.k[t] <= 0) continue;  // uniform
        const uint64_t th = a.state[t].prefix;
        uint64_t m[PR_CHUNK_ROUNDS];
#pragma unroll
        for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) m[r] = __ballot(ck[r] <= th);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) off[r * NW + wave] = (uint32_t)__popcll(m[r]);
        }
        __syncthreads();
        if (wave == 0) {
            const uint32_t v = off[lane];
            uint32_t incl = v;
#pragma unroll
            for (int o = 1; o < MGS_WAVE; o <<= 1) {
                const uint32_t y = (uint32_t)__shfl_up((int)incl, o, MGS_WAVE);
                if (lane >= o) incl += y;
            }
            off[lane] = a.cnt[(int64_t)t * a.nblk + blockIdx.x] + incl - v;
        }
        __syncthreads();
        int32_t* out = a.kept + a.koff[t];
#pragma unroll
        for (int r = 0; r < PR_CHUNK_ROUNDS; ++r) {
            if ((m[r] >> lane) & 1ull) {
                const uint32_t pos = off[r * NW + wave] + (uint32_t)__popcll(m[r] & lt_mask);
                if (pos < (uint64_t)a.k[t]) out[pos] = (int32_t)(base + r * PR_CHUNK_THREADS + threadIdx.x);
            }
        }
        __syncthreads();  // off is rewritten for the next ratio
    }
}

// Workspace layout.
struct PruneLayout {
    size_t state, hist0, histA, histB, cnt, total;
};

PruneLayout prune_layout(int64_t n, int32_t T) {
    PruneLayout L;
    size_t o = MGS_STATUS_BYTES;
    L.state = o;
    o += mgs_align_up(sizeof(PruneState) * MGS_MAX_RATIOS, 256);
    L.hist0 = o;
    o += sizeof(uint32_t) * PR_BINS;
    L.histA = o;
    o += sizeof(uint32_t) * PR_BINS * (size_t)std::max(T, 1);
    L.histB = o;
    o += sizeof(uint32_t) * PR_BINS * (size_t)std::max(T, 1);
    L.cnt = o;
    int64_t nblk = (n + PR_CHUNK - 1) / PR_CHUNK;
    o += mgs_align_up(sizeof(uint32_t) * (size_t)std::max<int64_t>(nblk, 1) * (size_t)std::max(T, 1), 256);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace mgs

extern "C" size_t mgs_prune_select_ws_bytes(int64_t n, int32_t T) {
    if (n < 0) n = 0;
    if (T < 1) T = 1;
    if (T > MGS_MAX_RATIOS) T = MGS_MAX_RATIOS;
    return mgs::prune_layout(n, T).total;
}

extern "C" int mgs_prune_select(const float* d_imp, int64_t n, const int64_t* h_k, int32_t T,
                                int32_t* d_kept, void* d_ws, size_t ws_bytes, void* stream) {
    using namespace mgs;
    if (n < 0 || n >= ((int64_t)1 << 31) || T < 1 || T > MGS_MAX_RATIOS || !h_k) return MGS_EINVAL;
    int64_t ksum = 0;
    for (int t = 0; t < T; ++t) {
        if (h_k[t] < 0 || h_k[t] > n) return MGS_EINVAL;
        ksum += h_k[t];
    }
    if (n > 0 && !d_imp) return MGS_EINVAL;
    if (ksum > 0 && !d_kept) return MGS_EINVAL;
    PruneLayout L = prune_layout(n, T);
    if (!d_ws || ws_bytes < L.total) return MGS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    PruneArgs a;
    std::memset(&a, 0, sizeof(a));
    a.imp = d_imp;
    a.status = (mgs_status_block*)ws;
    a.state = (PruneState*)(ws + L.state);
    a.hist0 = (uint32_t*)(ws + L.hist0);
    a.histA = (uint32_t*)(ws + L.histA);
    a.histB = (uint32_t*)(ws + L.histB);
    a.cnt = (uint32_t*)(ws + L.cnt);
    a.kept = d_kept;
    a.n = n;
    a.nblk = (n + PR_CHUNK - 1) / PR_CHUNK;
    a.T = T;
    int64_t off = 0;
    for (int t = 0; t < T; ++t) {
        a.k[t] = h_k[t];
        a.koff[t] = off;
        off += h_k[t];
    }
    int rc = mgs_fill<uint32_t>((uint32_t*)ws, 64, 0u, s);
    if (rc) return rc;
    rc = mgs_fill<uint32_t>(a.hist0, PR_BINS, 0u, s);
    if (rc) return rc;
    if (n == 0 || ksum == 0) return MGS_OK;
    int64_t hblocks = std::min<int64_t>((n + PR_HIST_THREADS * 16 - 1) / (PR_HIST_THREADS * 16), 2048);
    hipLaunchKernelGGL(prune_hist0_kernel, dim3((unsigned)hblocks), dim3(PR_HIST_THREADS), 0, s, a);
    hipLaunchKernelGGL(prune_select_kernel, dim3(T), dim3(256), 0, s, a, 0);
    for (int level = 1; level < PR_LEVELS; ++level) {
        hipLaunchKernelGGL(prune_hist_kernel, dim3((unsigned)hblocks), dim3(PR_HIST_THREADS), 0, s, a,
                           level);
        hipLaunchKernelGGL(prune_select_kernel, dim3(T), dim3(256), 0, s, a, level);
    }
    // ratios per compaction block: about 2048 blocks in all (enough to fill
    // the chip; more blocks would only read the same keys again)
    const int tb = (int)std::min<int64_t>(T, std::max<int64_t>(1, (T * a.nblk + 2047) / 2048));
    const unsigned tgroups = (unsigned)((T + tb - 1) / tb);
    hipLaunchKernelGGL(prune_count_kernel, dim3((unsigned)a.nblk, tgroups), dim3(PR_CHUNK_THREADS), 0, s, a, tb);
    hipLaunchKernelGGL(prune_scan_kernel, dim3(T), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(prune_write_kernel, dim3((unsigned)a.nblk, tgroups), dim3(PR_CHUNK_THREADS), 0, s, a, tb);
    return mgs_last_launch();
}
