// Nearest-codeword assignment of the vector quantizer for the higher-degree
// SH coefficients.  Paper: section "Attribute Transformation", clustering of
// the 1+D SH coefficients (a codebook plus an index mapping table, refined by
// mini-batch k-means whose inner step is this assignment).
//
// Definition: idx_i = argmin_j sum_d (x_id - c_jd)^2 with the distance summed
// in FP64 over d in order; ties -> smallest j.
//
// Method.  argmin_j ||x - c_j||^2 = argmin_j s_j with s_j = ||c_j||^2 - 2 x.c_j.
//   1. Scores s~_j from FP16 MFMA (v_mfma_f32_32x32x16_f16, FP32
//      accumulation) on the scaled vectors sigma x and sigma c, sigma a power
//      of two that puts the largest codeword norm cmax in [2^6, 2^7), so the
//      scores are sigma^2 s_j.  The codeword tile is the A operand (32
//      codewords x 16 dims), the X tile the B operand (16 dims x 32 rows), so
//      each lane owns one row and 16 codewords of every 32x32 output tile and
//      keeps its running minimum without cross-lane work.  ||sigma c_j||^2
//      enters as two extra K columns (its FP16 high and low parts) against
//      constant 1s in X.  A row with a scaled value of 2^15 or more (outside
//      FP16) goes to the exact scan of step 3.
//   2. Error bound per row, in scaled units (xs = sigma |x_i|, cs = sigma cmax):
//        E_i = (2u+u^2) xs 2cs + a(1+u) sqrt(D)(2cs + xs) + D a^2 + 2u^2 cs^2 + 2a
//              + g (2.02 xs cs + 1.01 cs^2)
//      (u = 2^-11 FP16 rounding, a = 2^-14 for values below the FP16 normal
//      range whether kept or flushed, g = (D+3) 2^-23 for any FP32
//      accumulation order).  The exact winner then satisfies
//      s~_j <= min s~ + 2 E_i; a small FP64 slack 2 delta_i also admits the
//      winner of the FP64 definition when exact distances tie within FP64
//      rounding.
//   3. One pass over the codebook.  Both lanes of a row keep the row's
//      running minimum m of the scores seen so far and record the tiles whose
//      smallest score (over the row's 32 codewords of the tile) is within T_i
//      of it; each lane stores a mask of its own codewords scoring at most
//      m + T_i (m taken after the tile; up to 8 tiles per lane, none when the
//      mask is empty).  A tile that lowers m so far that m + T_i falls below
//      the previous minimum clears the lists: every earlier recorded tile
//      scored at least that previous minimum, so above the final threshold
//      (the row minimum only falls), and cannot hold the winner.  Thresholds
//      only fall, so each mask holds every codeword under the final
//      threshold.  The row's candidates are then re-scored, two at a time,
//      with the FP64 definition (same operation order) and the smallest
//      (distance, index) wins.  Rows with more candidate tiles than slots go
//      to an exact FP64 full scan.  Padding codewords (up to whole chunks)
//      score +inf and never become candidates.
// The result equals the FP64 definition bit for bit.
//
// Layout.  The prepared codebook is stored chunk by chunk (64 codewords) as
// 16-byte units, unit-major: unit u of codeword r of a chunk sits at unit
// index u * 64 + r.  A chunk is one contiguous block (copied straight into
// LDS), and the 32 lanes that read one unit of 32 codewords read 512
// contiguous bytes, free of bank conflicts.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace mgs {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int VQ_WAVES = 4;
constexpr int VQ_THREADS = VQ_WAVES * MGS_WAVE;
constexpr int VQ_ROWSETS = 2;                          // 32-row sets per wave
constexpr int VQ_ROWS = VQ_WAVES * VQ_ROWSETS * 32;    // rows per workgroup
constexpr int VQ_CHUNK = 64;                           // codewords per LDS chunk (two buffers)
constexpr int VQ_CAND = 8;                             // candidate tiles per lane and row set

struct VqArgs {
    const float* x;
    const float* cb;
    int32_t* idx;
    double* dist;
    int64_t* nfb_out;
    mgs_status_block* status;
    _Float16* cbp;        // [Kpad][KP] prepared codebook (-2 sigma c, ||sigma c||^2 hi, lo, 0 pad)
    uint32_t* cmax_bits;  // max codeword norm, FP32 bits (rounded up)
    uint32_t* fb_count;
    int32_t* fb_list;
    int64_t N;
    int32_t D, K, Kpad, KP;
    int32_t xvec;         // D % 4 == 0 and x 16-byte aligned: rows load as float4
    int32_t cvec;         // D % 4 == 0 and the codebook 16-byte aligned: codewords load as float4
};

// The scale of the MFMA operands: 2^(6 - e) for cmax in [2^e, 2^(e+1)), so
// that |sigma c_j| < 2^7 and ||sigma c_j||^2 < 2^14 (1 for a zero or
// non-finite maximum).
__device__ __forceinline__ float vq_scale(float cm) {
    if (!(cm > 0.0f) || !finite_f32(cm)) return 1.0f;
    int ex;
    (void)frexpf(cm, &ex);  // cm = m 2^ex, m in [0.5, 1)
    return ldexpf(1.0f, min(max(7 - ex, -126), 126));
}

// The codeword-norm maximum, rounded up (the status word, the maximum and
// the fallback counter are cleared before this kernel).  One thread per
// codeword.
__global__ __launch_bounds__(256) void vq_norm_kernel(VqArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    float nrm = 0.0f;  // FP32 bits of non-negative floats order as unsigned ints
    if (j < a.K) {
        const float* c = a.cb + (int64_t)j * a.D;
        double n2 = 0.0;
        bool bad = false;
        for (int k = 0; k < a.D; ++k) {
            const float v = c[k];
            bad |= !finite_f32(v);
            n2 += (double)v * (double)v;
        }
        if (bad) atomicOr(&a.status->nonfinite, 1u);
        nrm = (float)sqrt(n2) * (1.0f + 1.0e-6f);
    }
    // the block's largest norm, then one atomic per block (thousands of
    // atomics on one address serialise)
    __shared__ uint32_t red[256 / MGS_WAVE];
    uint32_t m = __float_as_uint(nrm);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, MGS_WAVE));
    if ((threadIdx.x & (MGS_WAVE - 1)) == 0) red[threadIdx.x / MGS_WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / MGS_WAVE); ++w) m = max(m, red[w]);
        m = max(m, red[0]);
        atomicMax(a.cmax_bits, m);
    }
}

// Prepared codebook: -2 sigma c and the high and low FP16 parts of
// ||sigma c||^2 (FP64), zero padding.  Padding codewords (j >= K) are zero
// but for an infinite norm part: against the constant 1 of every X row they
// score +inf (the other products are 0 x finite), so they never lower a
// minimum nor pass a threshold.  One thread per codeword; the loops run over
// the compile-time row width, so the codeword's loads are all issued before
// use and its row is written as 16-byte units.
template <int KS>
__global__ __launch_bounds__(256) void vq_prep_kernel(VqArgs a) {
    constexpr int KP = 16 * KS;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.Kpad) return;
    // unit u of codeword j: chunk j / 64, unit-major inside the chunk
    f16x8* row = (f16x8*)(a.cbp + (int64_t)(j / VQ_CHUNK) * VQ_CHUNK * KP) + (j % VQ_CHUNK);
    if (j >= a.K) {
#pragma unroll
        for (int u = 0; u < KP / 8; ++u) {
            f16x8 w{};
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (8 * u + i == a.D) w[i] = (_Float16)INFINITY;
            row[u * VQ_CHUNK] = w;
        }
        return;
    }
    const float sg = vq_scale(__uint_as_float(*a.cmax_bits));
    const float* c = a.cb + (int64_t)j * a.D;
    float v[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) v[k] = k < a.D ? c[k] * sg : 0.0f;  // exact power-of-two scaling
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < KP; ++k)
        if (k < a.D) n2 += (double)v[k] * (double)v[k];
    const _Float16 hi = (_Float16)(float)n2;
    const _Float16 lo = (_Float16)(float)(n2 - (double)(float)hi);
#pragma unroll
    for (int u = 0; u < KP / 8; ++u) {
        f16x8 w;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * u + i;
            w[i] = k < a.D ? (_Float16)(-2.0f * v[k]) : k == a.D ? hi : k == a.D + 1 ? lo : (_Float16)0.0f;
        }
        row[u * VQ_CHUNK] = w;
    }
}

__device__ __forceinline__ double exact_dist(const float* __restrict__ x, const float* __restrict__ c,
                                             int D) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) {
        double d = (double)x[k] - (double)c[k];
        s += d * d;
    }
    return s;
}

// The distances of one row to two codewords, each the same terms added in
// the same order as above, from float4 loads: the row and both codewords are
// read in batches of four float4 groups, a batch's loads all issued before its
// first use (a group past D is read from the row's last group and ignored),
// and the two sums are independent chains.  Needs D % 4 == 0 and 16-byte
// aligned rows.
template <int NG>
__device__ __forceinline__ void exact_dist_vec2(const float* __restrict__ x, const float* __restrict__ c0,
                                                const float* __restrict__ c1, int D, double* d0, double* d1) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int g0 = 0; g0 < NG; g0 += 4) {
        if (4 * g0 >= D) break;
        float4 xv[4], av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k0 = 4 * (g0 + i) < D ? 4 * (g0 + i) : D - 4;
            xv[i] = *(const float4*)(x + k0);
            av[i] = *(const float4*)(c0 + k0);
            bv[i] = *(const float4*)(c1 + k0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float xe[4] = {xv[i].x, xv[i].y, xv[i].z, xv[i].w};
            const float ae[4] = {av[i].x, av[i].y, av[i].z, av[i].w};
            const float be[4] = {bv[i].x, bv[i].y, bv[i].z, bv[i].w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * (g0 + i) + e < D) {
                    const double xd = (double)xe[e];
                    const double da = xd - (double)ae[e];
                    const double db = xd - (double)be[e];
                    s0 += da * da;
                    s1 += db * db;
                }
        }
    }
    *d0 = s0;
    *d1 = s1;
}

template <int KS>
// Four waves per SIMD (at most 128 VGPRs) for D <= 46; wider rows take three.
__global__ __launch_bounds__(VQ_THREADS) __attribute__((amdgpu_waves_per_eu(KS <= 3 ? 4 : 3)))
void vq_main_kernel(VqArgs a) {
    constexpr int KP = 16 * KS;
    constexpr int UNITS = KP / 8;  // 16-byte units per prepared codeword
    // two chunk buffers, filled by direct global-to-LDS loads (64 lanes x 16
    // contiguous bytes per instruction, so the rows are not padded).  They are
    // two variables and every chunk step reads a fixed one, so the compiler
    // can tell that the copy into one buffer leaves the other alone and does
    // not wait for the copy before reading.
    __shared__ __attribute__((aligned(16))) _Float16 cbs0[VQ_CHUNK * KP];
    __shared__ __attribute__((aligned(16))) _Float16 cbs1[VQ_CHUNK * KP];
    // candidate tiles: tile index and the mask of the lane's codewords in it
    __shared__ int32_t cand_t[VQ_WAVES][VQ_ROWSETS][VQ_CAND][MGS_WAVE];
    __shared__ uint16_t cand_m[VQ_WAVES][VQ_ROWSETS][VQ_CAND][MGS_WAVE];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5;  // which 8 of each 16 dims / which 4-row blocks of the output
    const int D = a.D, K = a.K;
    const int64_t row0 = (int64_t)blockIdx.x * VQ_ROWS + wave * (VQ_ROWSETS * 32);

    // Asynchronous copy of chunk c0 of the prepared codebook into buffer
    // `dst`: wave w moves units [(i*VQ_WAVES + w)*64, +64) of the chunk; the
    // LDS base of each instruction is uniform over the wave.
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    auto prefetch = [&](int c0, _Float16* dst) {
        constexpr int nunits = VQ_CHUNK * UNITS;  // Kpad is a whole number of chunks
        const char* src = (const char*)(a.cbp + (int64_t)c0 * KP);
#pragma unroll
        for (int i = 0; i < (VQ_CHUNK * UNITS + VQ_THREADS - 1) / VQ_THREADS; ++i) {
            const int ublk = (i * VQ_WAVES + wave_u) * MGS_WAVE;
            if (ublk + lane < nunits)
                __builtin_amdgcn_global_load_lds(
                    (const void*)(src + (size_t)(ublk + lane) * 16),
                    (__attribute__((address_space(3))) void*)((char*)dst + ublk * 16), 16, 0, 0);
        }
    };
    // the first chunk's copy is under way while the rows are read and the
    // bounds computed
    prefetch(0, cbs0);

    // ---- B operands (the scaled X rows), bound T per row
    f16x8 breg[VQ_ROWSETS][KS];
    float T[VQ_ROWSETS];
    bool big[VQ_ROWSETS];  // a scaled value outside FP16: exact scan
    uint32_t bad = 0;
    const float cm = __uint_as_float(*a.cmax_bits);
    const float sg = vq_scale(cm);
#pragma unroll
    for (int rs = 0; rs < VQ_ROWSETS; ++rs) {
        const int64_t r = row0 + rs * 32 + (lane & 31);
        float n2 = 0.0f;
        bool bg = false;
        if (a.xvec) {
            // D % 4 == 0 and 16-byte aligned rows: every group of 4 dims is one
            // unconditional float4 load from an in-bounds address (row and
            // group clamped), all issued before any is used; values outside
            // the row (padding dims, rows past N) are then selected away
            const int64_t rr = r < a.N ? r : a.N - 1;
            float4 t[KS][2];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k0 = 16 * ks + 8 * half + 4 * h;
                    const int kk = k0 < D ? k0 : D - 4;
                    t[ks][h] = *(const float4*)(a.x + rr * D + kk);
                }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = 16 * ks + 8 * half + i;
                    const float4 q = t[ks][i >> 2];
                    const float e = (i & 3) == 0 ? q.x : (i & 3) == 1 ? q.y : (i & 3) == 2 ? q.z : q.w;
                    float v = 0.0f;
                    if (k < D) {
                        if (r < a.N) {
                            bad |= (uint32_t)!finite_f32(e);
                            n2 += e * e;
                            v = e * sg;
                            bg |= !(fabsf(v) < 32768.0f);
                        }
                    } else if (k == D || k == D + 1) {
                        v = 1.0f;  // every row, rows past N too (a padding codeword then scores +inf)
                    }
                    breg[rs][ks][i] = (_Float16)v;
                }
        } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = 16 * ks + 8 * half + i;
                    float v = 0.0f;
                    if (k < D) {
                        if (r < a.N) {
                            const float e = a.x[r * D + k];
                            bad |= (uint32_t)!finite_f32(e);
                            n2 += e * e;
                            v = e * sg;
                            bg |= !(fabsf(v) < 32768.0f);
                        }
                    } else if (k == D || k == D + 1) {
                        v = 1.0f;
                    }
                    breg[rs][ks][i] = (_Float16)v;
                }
            }
        }
        n2 += __shfl_xor(n2, 32, MGS_WAVE);
        big[rs] = (bg | (__shfl_xor((int)bg, 32, MGS_WAVE) != 0));
        // the bound in scaled units (sigma is a power of two)
        const double xs = (double)sg * (sqrt((double)n2) * (1.0 + 1.0e-5) + 1e-30);
        const double cs = (double)sg * (double)cm;
        const double u = 0x1p-11, aa = 0x1p-14, rd = sqrt((double)D);
        const double g = (double)(D + 3) * 0x1p-23;
        const double E = (2.0 * u + u * u) * xs * (2.0 * cs) + aa * (1.0 + u) * rd * (2.0 * cs + xs) +
                         (double)D * aa * aa + 2.0 * u * u * cs * cs + 2.0 * aa +
                         g * (2.02 * xs * cs + 1.01 * cs * cs);
        const double delta = 2.0 * (D + 2) * 0x1p-52 * (xs + cs) * (xs + cs);
        const double scale = cs * cs + 2.0 * xs * cs;
        T[rs] = (float)((2.0 * E + 2.0 * delta) * 1.0001 + 1.0e-6 * scale + 1e-30);
    }
    if (bad) atomicOr(&a.status->nonfinite, 1u);

    float mrun[VQ_ROWSETS];  // running minimum of the row's scores
    float mthr[VQ_ROWSETS];  // mrun + T, the recording threshold
    int cnt[VQ_ROWSETS];
#pragma unroll
    for (int rs = 0; rs < VQ_ROWSETS; ++rs) {
        mrun[rs] = INFINITY;
        mthr[rs] = mrun[rs] + T[rs];
        cnt[rs] = 0;
    }

    const int nchunks = a.Kpad / VQ_CHUNK;
    // Chunk step q reads buffer q % 2 while the next chunk is copied into the
    // other one.
    auto chunk = [&](int q, const _Float16* cb_l, _Float16* other) {
        const int c0 = q * VQ_CHUNK;
        // the other buffer was last read before the barrier that ended the
        // previous step: fill it with the next chunk while this one is
        // processed
        if (q + 1 < nchunks) prefetch(c0 + VQ_CHUNK, other);
        // scores of one 32-codeword tile for the wave's row sets; K steps
        // outer, row sets inner: consecutive MFMAs are independent.  Lane l
        // reads unit 2 ks + (l / 32) of codeword tile * 32 + l % 32: 512
        // contiguous bytes per half-wave
        auto scores = [&](int tile, f32x16 (&acc)[VQ_ROWSETS]) {
            f16x8 areg[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                areg[ks] = *(const f16x8*)((const char*)cb_l +
                                            (size_t)(((2 * ks + half) * VQ_CHUNK) + tile * 32 + (lane & 31)) * 16);
#pragma unroll
            for (int rs = 0; rs < VQ_ROWSETS; ++rs) acc[rs] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int rs = 0; rs < VQ_ROWSETS; ++rs)
                    acc[rs] = __builtin_amdgcn_mfma_f32_32x32x16_f16(areg[ks], breg[rs][ks], acc[rs], 0, 0, 0);
        };
        auto epilogue = [&](int tile, const f32x16 (&acc)[VQ_ROWSETS]) {
            const int jbase = c0 + tile * 32;
#pragma unroll
            for (int rs = 0; rs < VQ_ROWSETS; ++rs) {
                float sc[16];  // padding codewords score +inf
#pragma unroll
                for (int i = 0; i < 16; ++i) sc[i] = acc[rs][i];
                float tmin = sc[0];
#pragma unroll
                for (int i = 1; i < 16; ++i) tmin = fminf(tmin, sc[i]);
                // the row's smallest score in the tile: lanes l and l ^ 32 hold
                // its two halves (v_permlane32_swap exchanges the halves), so
                // both lanes of a row keep the same running minimum and decide
                // alike (half as many independent decisions per wavefront)
                {
                    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(tmin), __float_as_uint(tmin),
                                                                     false, false);
                    tmin = fminf(tmin, fminf(__uint_as_float(sw[0]), __uint_as_float(sw[1])));
                }
                if (!(tmin <= mthr[rs])) continue;  // most row-tiles hold no candidate
                const float mo = mrun[rs];
                mrun[rs] = fminf(mo, tmin);
                const float thr = mrun[rs] + T[rs];
                mthr[rs] = thr;
                if (thr < mo) cnt[rs] = 0;  // no earlier tile can hold the winner
                // sign bits of thr - s, shifted in by v_alignbit (element i
                // lands in bit 15 - i); s <= thr  <=>  thr - s >= 0 (an exact
                // zero difference is +0), so the mask is the complement
                uint32_t neg = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    neg = __builtin_amdgcn_alignbit(neg, __float_as_uint(thr - sc[i]), 31);
                const uint32_t bits = ~neg & 0xFFFFu;
                if (bits == 0u) continue;  // this lane's half of the tile holds none
                if (cnt[rs] < VQ_CAND) {
                    cand_t[wave][rs][cnt[rs]][lane] = jbase;
                    cand_m[wave][rs][cnt[rs]][lane] = (uint16_t)bits;
                }
                cnt[rs] += 1;  // a count past VQ_CAND marks the overflow
            }
        };
        // software pipeline: the next tile's MFMAs are issued before this
        // tile's epilogue, so the matrix cores work while the VALU does
        // (two accumulator sets, alternating)
        constexpr int ntiles = VQ_CHUNK / 32;
        f32x16 acc0[VQ_ROWSETS], acc1[VQ_ROWSETS];
        scores(0, acc0);
        int tile = 0;
        for (; tile + 2 < ntiles; tile += 2) {
            scores(tile + 1, acc1);
            epilogue(tile, acc0);
            scores(tile + 2, acc0);
            epilogue(tile + 1, acc1);
        }
        if (tile + 1 < ntiles) {
            scores(tile + 1, acc1);
            epilogue(tile, acc0);
            epilogue(tile + 1, acc1);
        } else {
            epilogue(tile, acc0);
        }
        // the step's MFMAs are issued before the wait (the scheduler would
        // otherwise hoist the wait over them and expose the copy's latency)
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);  // this wave's part of the next chunk has landed
        __syncthreads();                // ... and everyone's; this buffer is free
    };
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // step q reads buffer q % 2
    int q = 0;
    for (; q + 1 < nchunks; q += 2) {
        chunk(q, cbs0, cbs1);
        chunk(q + 1, cbs1, cbs0);
    }
    if (q < nchunks) chunk(q, cbs0, cbs1);

    // ---- exact FP64 re-rank of the row's candidates (both lanes of the row)
#pragma unroll
    for (int rs = 0; rs < VQ_ROWSETS; ++rs) {
        const int64_t r = row0 + rs * 32 + (lane & 31);
        const int ovf = cnt[rs] > VQ_CAND || big[rs];
        const int ovf_row = ovf | __shfl_xor(ovf, 32, MGS_WAVE);
        double best = INFINITY;
        int32_t bj = 0x7fffffff;
        if (r < a.N && !ovf_row) {
            const float* xr = a.x + r * D;
            const bool vec = a.xvec && a.cvec;  // float4 rows and codewords
            int e = 0;
            int jbase = cnt[rs] > 0 ? cand_t[wave][rs][0][lane] : 0;
            uint32_t bits = cnt[rs] > 0 ? cand_m[wave][rs][0][lane] : 0u;
            // the lane's next candidate codeword; false once none is left
            auto next = [&](int32_t& j) {
                for (;;) {
                    while (bits) {
                        const int i = 15 - __builtin_ctz(bits);  // bit 15 - i holds element i
                        bits &= bits - 1;
                        // output element i of this lane: codeword row 8*(i/4) + 4*half + i%4
                        j = jbase + 8 * (i >> 2) + 4 * half + (i & 3);
                        if (j < K) return true;
                    }
                    if (++e >= cnt[rs]) return false;
                    jbase = cand_t[wave][rs][e][lane];
                    bits = cand_m[wave][rs][e][lane];
                }
            };
            auto take = [&](int32_t j, double d) {
                if (d < best || (d == best && j < bj)) {
                    best = d;
                    bj = j;
                }
            };
            // candidates in pairs (an odd last one is scored twice)
            int32_t j0 = 0, j1 = 0;
            bool more = next(j0);
            while (more) {
                if (!next(j1)) {
                    j1 = j0;
                    more = false;
                }
                const float* c0 = a.cb + (int64_t)j0 * D;
                const float* c1 = a.cb + (int64_t)j1 * D;
                double d0, d1;
                if (vec) {
                    exact_dist_vec2<KP / 4>(xr, c0, c1, D, &d0, &d1);
                } else {
                    d0 = exact_dist(xr, c0, D);
                    d1 = exact_dist(xr, c1, D);
                }
                take(j0, d0);
                take(j1, d1);
                if (more) more = next(j0);
            }
        }
        const double ob = __shfl_xor(best, 32, MGS_WAVE);
        const int32_t oj = __shfl_xor(bj, 32, MGS_WAVE);
        if (ob < best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
        if (r < a.N && half == 0) {
            if (ovf_row) {
                a.fb_list[atomicAdd(a.fb_count, 1u)] = (int32_t)r;
            } else {
                a.idx[r] = bj;
                if (a.dist) a.dist[r] = best;
            }
        }
    }
}

// Exact FP64 full scan for the rows whose candidate buffer overflowed: one
// workgroup per row (all four waves stride over the codewords, then the
// smallest (distance, index) over the workgroup), rows strided over the grid.
__global__ __launch_bounds__(256) void vq_fallback_kernel(VqArgs a) {
    __shared__ double wbest[4];
    __shared__ int32_t wj[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t total = *a.fb_count;
    if (a.nfb_out && blockIdx.x == 0 && threadIdx.x == 0) *a.nfb_out = (int64_t)total;
    for (int64_t i = blockIdx.x; i < total; i += gridDim.x) {  // uniform over the workgroup
        const int32_t r = a.fb_list[i];
        const float* xr = a.x + (int64_t)r * a.D;
        double best = INFINITY;
        int32_t bj = 0x7fffffff;
        for (int j = threadIdx.x; j < a.K; j += 256) {
            const double d = exact_dist(xr, a.cb + (int64_t)j * a.D, a.D);
            if (d < best) {  // j increases per thread: strict < keeps the smallest j
                best = d;
                bj = j;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(best, o, MGS_WAVE);
            const int32_t oj = __shfl_xor(bj, o, MGS_WAVE);
            if (ob < best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (lane == 0) {
            wbest[wave] = best;
            wj[wave] = bj;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w)
                if (wbest[w] < best || (wbest[w] == best && wj[w] < bj)) {
                    best = wbest[w];
                    bj = wj[w];
                }
            a.idx[r] = bj;
            if (a.dist) a.dist[r] = best;
        }
        __syncthreads();
    }
}

struct VqLayout {
    size_t cmax, cbp, fb, total;
    int KS, KP, Kpad;
};

VqLayout vq_layout(int64_t N, int D, int K) {
    VqLayout L;
    L.KS = (D + 2 + 15) / 16;
    L.KP = 16 * L.KS;
    // whole chunks: padding codewords score +inf in the main kernel
    L.Kpad = (int)(((int64_t)K + VQ_CHUNK - 1) / VQ_CHUNK * VQ_CHUNK);
    size_t o = MGS_STATUS_BYTES;
    L.cmax = o;
    o += 256;
    L.cbp = o;
    o += mgs_align_up(sizeof(_Float16) * (size_t)L.Kpad * L.KP, 256);
    L.fb = o;
    o += mgs_align_up(sizeof(int32_t) * (size_t)std::max<int64_t>(N, 1), 256);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace mgs

extern "C" size_t mgs_vq_assign_ws_bytes(int64_t N, int32_t D, int32_t K) {
    if (N < 0 || D < 1 || D > MGS_MAX_VQ_DIM || K < 1 || K > (1 << 30)) return 0;
    return mgs::vq_layout(N, D, K).total;
}

extern "C" int mgs_vq_assign(const float* d_x, int64_t N, int32_t D, const float* d_cb, int32_t K,
                             int32_t* d_idx, double* d_dist, int64_t* d_nfallback, void* d_ws,
                             size_t ws_bytes, void* stream) {
    using namespace mgs;
    if (N < 0 || N >= ((int64_t)1 << 31) || D < 1 || D > MGS_MAX_VQ_DIM || K < 1 || K > (1 << 30) || !d_cb)
        return MGS_EINVAL;
    if (N > 0 && (!d_x || !d_idx)) return MGS_EINVAL;
    VqLayout L = vq_layout(N, D, K);
    if (!d_ws || ws_bytes < L.total) return MGS_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    VqArgs a;
    std::memset(&a, 0, sizeof(a));
    a.x = d_x;
    a.cb = d_cb;
    a.idx = d_idx;
    a.dist = d_dist;
    a.nfb_out = d_nfallback;
    a.status = (mgs_status_block*)ws;
    a.cmax_bits = (uint32_t*)(ws + L.cmax);
    a.fb_count = (uint32_t*)(ws + L.cmax + 64);
    a.cbp = (_Float16*)(ws + L.cbp);
    a.fb_list = (int32_t*)(ws + L.fb);
    a.N = N;
    a.D = D;
    a.K = K;
    a.Kpad = L.Kpad;
    a.KP = L.KP;
    a.xvec = (D % 4 == 0) && ((uintptr_t)d_x % 16 == 0);
    a.cvec = (D % 4 == 0) && ((uintptr_t)d_cb % 16 == 0);
    int rc = mgs_fill<uint32_t>((uint32_t*)ws, 64, 0u, s);       // status word
    if (rc) return rc;
    rc = mgs_fill<uint32_t>(a.cmax_bits, 64, 0u, s);              // norm maximum + fallback count
    if (rc) return rc;
    hipLaunchKernelGGL(vq_norm_kernel, dim3((K + 255) / 256), dim3(256), 0, s, a);
    const dim3 pgrid((L.Kpad + 255) / 256);
    switch (L.KS) {
        case 1: hipLaunchKernelGGL(vq_prep_kernel<1>, pgrid, dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL(vq_prep_kernel<2>, pgrid, dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL(vq_prep_kernel<3>, pgrid, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(vq_prep_kernel<4>, pgrid, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(vq_prep_kernel<5>, pgrid, dim3(256), 0, s, a); break;
    }
    if (N > 0) {
        const unsigned blocks = (unsigned)((N + VQ_ROWS - 1) / VQ_ROWS);
        switch (L.KS) {
            case 1: hipLaunchKernelGGL(vq_main_kernel<1>, dim3(blocks), dim3(VQ_THREADS), 0, s, a); break;
            case 2: hipLaunchKernelGGL(vq_main_kernel<2>, dim3(blocks), dim3(VQ_THREADS), 0, s, a); break;
            case 3: hipLaunchKernelGGL(vq_main_kernel<3>, dim3(blocks), dim3(VQ_THREADS), 0, s, a); break;
            case 4: hipLaunchKernelGGL(vq_main_kernel<4>, dim3(blocks), dim3(VQ_THREADS), 0, s, a); break;
            default: hipLaunchKernelGGL(vq_main_kernel<5>, dim3(blocks), dim3(VQ_THREADS), 0, s, a); break;
        }
    }
    hipLaunchKernelGGL(vq_fallback_kernel, dim3(2048), dim3(256), 0, s, a);
    return mgs_last_launch();
}
