// Group-wise quantization sweep: loss and entropy-size tables for every
// (reserve ratio, channel, group, candidate bit-width).
//
// Quantizer (paper, section "Group-wise Attribute Quantization"):
//   S = (max - min) / 2^b,  Z = round(2^b - max / S),
//   q = round(clamp(x / S + Z, 0, 2^b - 1)),  xhat = (q - Z) * S.
// Loss table (section "Acceleration"): importance-weighted sum of squared
// errors per group and b.  Size table (section "Size Estimator"): Shannon
// bound n * H of the group's codes, in bits.
//
// One workgroup owns one tile (ratio t, group g, a run of channels).  Per
// channel it gathers the group's values and weights into registers, reduces
// min / max, and then evaluates every candidate b from those registers:
// quantize, dequantize, error, and an LDS histogram of the codes.
// Histograms are laid out in LDS per "batch" of bit-widths that fit
// together; a b whose 2^b bins exceed the LDS capacity is split into bin
// windows counted in separate passes.  Bins are 32-bit counters, or two
// 16-bit counters per word where that is needed to fit (counts never exceed
// G <= 65535).  Histograms with few bins keep up to 32 lane-interleaved
// copies of every bin, so that the many lanes of a wavefront that land in
// one bin do not serialise on one LDS address; the scan adds the copies.
//
// Bit exactness of the codes.  The quantizer is evaluated with single FP32
// operations, round-half-even, no contraction (built -ffp-contract=off) and
// IEEE denormals.  Two exact rewrites save work per element and b:
//   1. x / S_b == (x / R) * 2^b whenever S_b = R * 2^-b is normal for every
//      listed b: S_b is then an exact power-of-two scaling of R, and
//      rounding commutes with such scalings while results stay normal;
//      a subnormal x / R only occurs for values far below the step and
//      leaves the code unchanged (it is absorbed by Z or rounds to 0).
//      fl(fl(x/S) + Z) is then one fma(x/R, 2^b, Z).  Groups that fail the
//      test (R < 2^(bmax - 126)) use the literal division per element.
//      x / R itself takes one reciprocal per group and two corrections by
//      the FMA remainder per element, which give the correctly rounded
//      quotient (see the quotients of the kernel).
//   2. round(clamp(t, 0, 2^b - 1)) == clamp(fl(t + 2^23), 2^23, 2^23 + 2^b - 1)
//      - 2^23: adding 2^23 rounds any t in [0, 2^23) to an integer
//      half-even, the clamp bounds are integers and fl() is monotone.  With
//      |Z| <= 2^23, fl(q - Z) is fl((t' ) - (2^23 + Z)) because both
//      operands are exact.
// Loss.  On those fast groups the values and steps are scaled by 2^-E with
// 2^E <= R < 2^(E+1); both scalings are exact, so the FP32 dequantized value
// is exactly xhat * 2^-E and every difference stays far from FP32 overflow.
// Each thread forms d = fl(xhat' - x'), and sums w * d^2 over its <= EPT
// elements in FP32; a fixed-order FP32 reduction over the wavefront follows
// (relative error <= (EPT + 9) * 2^-24 for these nonnegative terms), then
// the rescaling by 2^(2E) and an FP64 sum over waves, so results are
// deterministic.  A wave total that is not finite, or so small that
// underflowed terms could matter (below (W + 1) * 2^-112, W the largest
// weight of the group), is recomputed from the registers with FP64 terms.
// Literal-division groups and underflowed steps keep exact FP64 terms.
// Size.  n log2 n - sum_k h_k log2 h_k in FP64.  Scanned histograms take
// h log2 h per bin (LDS table for h < 256).  Histograms with more bins than
// a sixteenth of the group instead add, per element, the increment of its bin's old
// count c (returned by the atomic): F[c] = R(T(c+1)) - R(T(c)) with
// T(h) = h log2 h and R the rounding to a 2^-K grid, so a bin's increments
// telescope to R(T(h)) exactly and in any order.  The LDS copy of F covers
// c < 256 and is indexed by c mod 256; a bin that ends with h > 256 has
// then collected floor(h / 256) * R(T(256)) + R(T(h mod 256)), which a
// correction scan replaces by R(T(h)) (exact: all terms lie on the grid).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "sweep.h"

namespace mgs {

// h * log2(h) of a bin count (scanned histograms): small counts from the
// LDS copy, larger ones from the workspace table.  The two tables are read
// through pointers typed with their address spaces: a choice between two
// generic pointers becomes one flat load, which waits out the latency of
// global memory on every call.
__device__ __forceinline__ double hlog2h(uint32_t h, const double* lg, const double* lgt) {
    typedef const __attribute__((address_space(3))) double lds_f64;
    typedef const __attribute__((address_space(1))) double glb_f64;
    double v = ((lds_f64*)lg)[h < (uint32_t)LGTAB ? h : 0u];
    if (h >= (uint32_t)LGTAB) v = ((glb_f64*)lgt)[h];
    return v;
}

// FP64 value of a per-element FP32 copy.  The empty asm keeps the compiler
// from hoisting the conversion out of the bit-width loop, which would hold a
// second, FP64 copy of every element in registers.
__device__ __forceinline__ double as_f64(float v) {
    asm volatile("" : "+v"(v));
    return (double)v;
}

// Rounds to the grid 2^-K on which the entropy increments live.
__device__ __forceinline__ double grid_round(double v, int K) {
    return ldexp(rint(ldexp(v, K)), -K);
}

// Partial sums of one evaluation pass in one thread: the loss in FP32 (fast
// paths, values scaled by 2^-E, so the terms stay far from FP32 overflow and
// underflow) or in FP64 (literal-division and underflowed-step paths), and
// the entropy increments (FP64, exact grid sum).
struct Part {
    float err;
    double err64;
    double ent;
};

// Entropy increment of one more element in a bin whose counter read c
// before (the low 8 bits index the LDS table; the caller tracks larger
// counts for the correction scan).
__device__ __forceinline__ void add_increment(uint32_t c, const double* lf, Part& acc) {
    acc.ent += lf[c & (uint32_t)(LGTAB - 1)];
}

// Counter bits that reveal a count of 256 or more: every 16-bit half of a
// packed word, or the whole word.
__device__ __forceinline__ uint32_t big_count_mask(bool packed) {
    return packed ? 0xFF00FF00u : 0xFFFFFF00u;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// A pointer into the constant address space (global memory the kernel only
// reads and nothing writes while it runs).
template <typename T>
using constant_ptr = const __attribute__((address_space(4))) T*;
// A pointer into global memory.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

// LDS byte address of a shared-memory word (LDS addresses are 32-bit).
__device__ __forceinline__ uint32_t lds_addr(const uint32_t* p) {
    return (uint32_t)(uintptr_t)(const lds_u32*)p;
}

// Atomic add to the LDS word at byte address `addr`; returns the old value.
__device__ __forceinline__ uint32_t lds_add(uint32_t addr, uint32_t v) {
    return __hip_atomic_fetch_add((lds_u32*)(uintptr_t)addr, v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One histogram pass over the tile's elements for one bit-width on the fast
// path (x / S_b from x / R, 2^23 rounding trick), specialised on packed bins,
// ragged group, incremental entropy (RTN: the atomic's old count c gives
// the entropy increment F[c]; no scan of the bins afterwards), replicated
// bins, a bin window and whether the pass also sums the loss.
// xv holds x * 2^-E and Ss = S * 2^-E: both scalings are exact, so the
// dequantized value (q - Z) * Ss is exactly xhat * 2^-E.
// Bin addresses come straight from the bits of tm = 2^23 + q, which are
// 0x4B000000 + q: with the per-entry constant cadj (LDS base of the bins,
// replica lane, minus the shifted 0x4B000000; kept opaque so that the
// compiler does not re-associate it) the byte address of bin word
// (q << rl) | cpy is (bits << (rl + 2)) + cadj, one shift-add; packed bins
// (word q >> 1, half q & 1) use ((bits << 1) + cadj) & ~3 and the half's
// shift 16 * (q & 1) = (bits << 4) mod 32.
// REPL: 2^rl copies of every bin, bin q of lane l in word (q << rl) | cpy with
// cpy = l mod 2^rl, so lanes that share a bin hit different LDS banks.
// WIN: only the words at byte addresses [wlo, wlo + wbytes) live in LDS this
// pass; elements past the ragged end carry w = 0 and x = 0, so they add
// nothing to the loss.
// Returns the OR of the counters the pass read (RTN) in `seen`.
template <int NT, int EPT, bool PACKED, bool CHECK, bool RTN, bool REPL, bool WIN, bool ERR>
__device__ __forceinline__ Part eval_fast(const float (&u)[EPT], const float (&xv)[EPT],
                                          const float (&wv)[EPT], int n, int tid, float P, float Ss,
                                          float Z, uint32_t cadj, uint32_t wlo, uint32_t wbytes, int rl,
                                          const double* lf, uint32_t& seen) {
    const float M = 8388608.0f;  // 2^23
    const float MZ = M + Z;
    const float hi = M + (P - 1.0f);
    const uint32_t shl = REPL ? (uint32_t)rl + 2u : 2u;
    Part acc{0.0f, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const bool valid = !CHECK || i * NT + tid < n;
        if (!WIN && !valid) continue;
        float t = __builtin_fmaf(u[i], P, Z);
        float tm = __builtin_amdgcn_fmed3f(t + M, M, hi);
        const uint32_t tb = __float_as_uint(tm);
        uint32_t addr, inc = 1u, sh = 0u;
        if (PACKED) {
            addr = ((tb << 1) + cadj) & ~3u;
            sh = (tb << 4) & 31u;
            inc = 1u << sh;
        } else {
            addr = (tb << shl) + cadj;
        }
        if (!WIN || (valid && addr - wlo < wbytes)) {
            const uint32_t old = lds_add(addr, inc);
            if (RTN) {
                acc.ent += lf[PACKED ? __builtin_amdgcn_ubfe(old, sh, 8) : (old & (uint32_t)(LGTAB - 1))];
                seen |= old;
            }
        }
        if (ERR) {
            float xh = (tm - MZ) * Ss;
            float d = xh - xv[i];
            acc.err = __builtin_fmaf(wv[i], d * d, acc.err);
        }
    }
    return acc;
}

// The same pass for the rare cases, with runtime switches: |Z| > 2^23 (rint
// path) or the literal division per element, bins possibly in windows.
// Literal tiles are never scaled (E = 0, Ss = S) and keep the loss in FP64.
template <int NT, int EPT>
__device__ __forceinline__ Part eval_generic(const float (&u)[EPT], const float (&xv)[EPT],
                                             const float (&wv)[EPT], int n, int tid, float P, float S,
                                             float Ss, float Z, uint32_t* hist, int base, int lo,
                                             int nwords, bool packed, int rl, int cpy, bool literal,
                                             bool err, bool rtn, const double* lf, uint32_t& seen) {
    const float qmax = P - 1.0f;
    Part acc{0.0f, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        if (i * NT + tid >= n) continue;
        float t;
        if (literal) {
            t = xv[i] / S;
            t = t + Z;
        } else {
            t = __builtin_fmaf(u[i], P, Z);
        }
        t = __builtin_amdgcn_fmed3f(t, 0.0f, qmax);
        float q = __builtin_rintf(t);
        uint32_t qi = (uint32_t)q;
        int word = packed ? (int)(qi >> 1) : (((int)qi << rl) | cpy);
        uint32_t sh = packed ? ((qi & 1u) << 4) : 0u;
        if ((uint32_t)(word - lo) < (uint32_t)nwords) {
            uint32_t old = atomicAdd(&hist[base + word], 1u << sh);
            if (rtn) {
                add_increment(old >> sh, lf, acc);
                seen |= old;
            }
        }
        if (err) {
            float xh = (q - Z) * Ss;
            if (literal) {
                double d = (double)xh - as_f64(xv[i]);
                acc.err64 = __builtin_fma(as_f64(wv[i]), d * d, acc.err64);
            } else {
                float d = xh - xv[i];
                acc.err = __builtin_fmaf(wv[i], d * d, acc.err);
            }
        }
    }
    return acc;
}

// FP64 loss of one non-literal pass, recomputed from the registers (the same
// codes and FP32 dequantized values as the pass, exact FP64 differences);
// used when the FP32 sum of a wavefront cannot be trusted.
template <int NT, int EPT>
__device__ __forceinline__ double loss_f64(const float (&u)[EPT], const float (&xv)[EPT],
                                        const float (&wv)[EPT], int n, int tid, float P, float Ss,
                                        float Z) {
    const float qmax = P - 1.0f;
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        if (i * NT + tid >= n) continue;
        float t = __builtin_amdgcn_fmed3f(__builtin_fmaf(u[i], P, Z), 0.0f, qmax);
        float xh = (__builtin_rintf(t) - Z) * Ss;
        double d = (double)xh - (double)xv[i];
        e = __builtin_fma((double)wv[i], d * d, e);
    }
    return e;
}

template <int NT, int EPT, bool PACKED>
__device__ __forceinline__ Part eval_fast_dispatch(bool check, bool rtn, bool win, bool err,
                                                   uint32_t cadj, uint32_t wlo, uint32_t wbytes, int rl,
                                                   const float (&u)[EPT], const float (&xv)[EPT],
                                                   const float (&wv)[EPT], int n, int tid, float P,
                                                   float Ss, float Z, const double* lf, uint32_t& seen) {
#define MGS_EVAL(CHK, RT, RP, WN, ER)                                                              \
    eval_fast<NT, EPT, PACKED, CHK, RT, RP, WN, ER>(u, xv, wv, n, tid, P, Ss, Z, cadj, wlo, wbytes, \
                                                    rl, lf, seen)
    if constexpr (PACKED) {
        // bin windows only occur on packed histograms; the loss is summed in
        // the first window of a bit-width
        if (win) {
            if (check) {
                if (rtn) return err ? MGS_EVAL(true, true, false, true, true) : MGS_EVAL(true, true, false, true, false);
                return err ? MGS_EVAL(true, false, false, true, true) : MGS_EVAL(true, false, false, true, false);
            }
            if (rtn) return err ? MGS_EVAL(false, true, false, true, true) : MGS_EVAL(false, true, false, true, false);
            return err ? MGS_EVAL(false, false, false, true, true) : MGS_EVAL(false, false, false, true, false);
        }
        if (check) return rtn ? MGS_EVAL(true, true, false, false, true) : MGS_EVAL(true, false, false, false, true);
        return rtn ? MGS_EVAL(false, true, false, false, true) : MGS_EVAL(false, false, false, false, true);
    } else {
        // replicated bins only ever appear on scanned (non-incremental) entries
        if (check) {
            if (rtn) return MGS_EVAL(true, true, false, false, true);
            return rl ? MGS_EVAL(true, false, true, false, true) : MGS_EVAL(true, false, false, false, true);
        }
        if (rtn) return MGS_EVAL(false, true, false, false, true);
        return rl ? MGS_EVAL(false, false, true, false, true) : MGS_EVAL(false, false, false, false, true);
    }
#undef MGS_EVAL
}

// Sum of v over each group of 2^rl adjacent lanes (rl <= 5), in the group's
// last lane: a sliding window built from DPP row shifts (lanes shifted in
// from outside the row read 0), then, for groups of 32, the row's window
// plus the previous row's (row broadcast of lane 15).  Other lanes hold
// partial sums.  Called by all lanes of a wave.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t v, int rl) {
    if (rl >= 1) v += dpp_u32<0x111, 0xF>(v);  // row_shr:1
    if (rl >= 2) v += dpp_u32<0x112, 0xF>(v);  // row_shr:2
    if (rl >= 3) v += dpp_u32<0x114, 0xF>(v);  // row_shr:4
    if (rl >= 4) v += dpp_u32<0x118, 0xF>(v);  // row_shr:8
    if (rl >= 5) v += dpp_u32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    return v;
}

// Wavefront min / max / OR by DPP row shifts and row broadcasts (lanes whose
// source lies outside the row, or rows the mask leaves out, take the
// identity); the result is read from lane 63, so every lane gets it.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_keep(uint32_t v, uint32_t ident) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <typename F>
__device__ __forceinline__ uint32_t wave_reduce_dpp(uint32_t v, uint32_t ident, F op) {
    v = op(v, dpp_keep<0x111, 0xF>(v, ident));
    v = op(v, dpp_keep<0x112, 0xF>(v, ident));
    v = op(v, dpp_keep<0x114, 0xF>(v, ident));
    v = op(v, dpp_keep<0x118, 0xF>(v, ident));
    v = op(v, dpp_keep<0x142, 0xA>(v, ident));
    v = op(v, dpp_keep<0x143, 0xC>(v, ident));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ float wave_min_dpp(float v) {
    return __uint_as_float(wave_reduce_dpp(__float_as_uint(v), __float_as_uint(INFINITY), [](uint32_t a, uint32_t b) {
        return __float_as_uint(fminf(__uint_as_float(a), __uint_as_float(b)));
    }));
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    return __uint_as_float(wave_reduce_dpp(__float_as_uint(v), __float_as_uint(-INFINITY), [](uint32_t a, uint32_t b) {
        return __float_as_uint(fmaxf(__uint_as_float(a), __uint_as_float(b)));
    }));
}
__device__ __forceinline__ uint32_t wave_or_dpp(uint32_t v) {
    return wave_reduce_dpp(v, 0u, [](uint32_t a, uint32_t b) { return a | b; });
}

// Waves per SIMD the register budget must allow: <= 128 VGPRs for shapes
// that hold 16 or fewer elements per thread, so that two 512-thread blocks
// (or four of 256) share a CU when their histograms fit in LDS.
template <int NT, int EPT, bool CHUNKED>
constexpr int sweep_min_waves() { return (EPT <= 16 && !CHUNKED) ? 4 : 1; }

template <int NT, int EPT, bool CHUNKED>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<NT, EPT, CHUNKED>())))
void sweep_kernel(SweepParams p) {
    constexpr int NW = NT / MGS_WAVE;
    extern __shared__ __align__(16) uint32_t hist[];  // 16-byte aligned: cleared and read as uint4
    __shared__ double lg[LGTAB];
    __shared__ double lf[LGTAB];
    __shared__ double errpart[MGS_MAX_BITS][NW];
    __shared__ double bitpart[MGS_MAX_BITS][NW];
    __shared__ float red_mn[NW], red_mx[NW], red_w[NW];
    __shared__ uint32_t red_bad[NW];
    __shared__ float prmS[MGS_MAX_BITS], prmZ[MGS_MAX_BITS];
    __shared__ uint32_t ovf_flag[MGS_MAX_ENTRIES];  // per batch: some bin passed the LDS increment table

    const int tid = threadIdx.x;
    const int lane = tid & (MGS_WAVE - 1);
    // the same in every lane of a wavefront: scalar, so that addresses made
    // from it are never held (or spilled) per lane
    const int wave = __builtin_amdgcn_readfirstlane(tid / MGS_WAVE);

    const double* __restrict__ lgt = p.lgtab;
    const double* __restrict__ lft = p.lgtab + (p.lgtab_max + 1);
    const uint32_t hist_lds = lds_addr(hist);
    for (int h = tid; h < LGTAB; h += NT) {
        lg[h] = h <= p.lgtab_max ? lgt[h] : 0.0;
        lf[h] = h <= p.lgtab_max ? lft[h] : 0.0;
    }
    // grid value of T(LGTAB), what one full cycle of the LDS increments adds
    // up to (only counts above LGTAB need it)
    const double rt_cycle = p.lgtab_max >= LGTAB ? grid_round(lgt[LGTAB], p.kgrid) : 0.0;

    // Workgroups are dispatched round-robin over the XCDs: each XCD gets a
    // contiguous run of tiles, so that one XCD's L2 serves the neighbouring
    // groups of every ratio.  A grid of one workgroup per tile strides over
    // its run (a grid that is not a multiple of the XCD count strides
    // plainly).  A persistent grid (p.persist: about one workgroup per
    // resident slot) takes tiles from a counter per run, in order, and when
    // its own XCD's run is drained moves on to the other runs; every counter
    // only grows, so each workgroup leaves once all runs are drained.
    const int64_t per = (p.ntiles + MGS_XCDS - 1) / MGS_XCDS;
    int64_t it0 = blockIdx.x, step = gridDim.x, it_end = p.ntiles;
    if (gridDim.x % MGS_XCDS == 0) {
        const int x = (int)(blockIdx.x % MGS_XCDS);
        it0 = (int64_t)x * per + blockIdx.x / MGS_XCDS;
        step = gridDim.x / MGS_XCDS;
        it_end = min(p.ntiles, (int64_t)(x + 1) * per);
    }
    __shared__ int64_t grabbed;
    const int qx0 = (int)(blockIdx.x % MGS_XCDS);
    int qk = 0;
    for (int64_t it = it0 - step;;) {
        if (p.persist) {
            bool got = false;
            while (qk < MGS_XCDS) {
                const int x = (qx0 + qk) % MGS_XCDS;
                const int64_t hi = min(p.ntiles, (int64_t)(x + 1) * per);
                if (tid == 0)
                    grabbed = (int64_t)x * per +
                              (int64_t)__hip_atomic_fetch_add(&p.status->queue[x], 1u, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                {  // the same value in every lane: keep it (and all that derives from it) scalar
                    const int64_t g = grabbed;
                    it = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(g >> 32)) << 32) |
                                   (uint32_t)__builtin_amdgcn_readfirstlane((int)g));
                }
                __syncthreads();  // every thread has read it before the next grab
                if (it < hi) {
                    got = true;
                    break;
                }
                ++qk;
            }
            if (!got) break;
        } else {
            it += step;
            if (it >= it_end) break;
        }
        // ---- locate the tile: scene, then (channel run, ratio t, group g)
        // with the run's groups taken in the scene's tile order; channels
        // [c0, c1)
        int sid = 0;
        int64_t rank;
        int part = -1;  // split tail: the channel run of a split group (-1: the whole group)
        int cc = 0;     // plain tiles: the channel run
        if (p.tsplit) {
            // All channels per tile, persistent grid: the scenes' groups in one
            // sequence (scene by scene, each in its tile order; tcum holds the
            // prefix of the groups).  XCD x's counter range holds the groups
            // [x gpx, (x+1) gpx) of it, the first ones whole and the last
            // tranks of them in tparts channel runs of tcpb channels each, so
            // that the range ends in small tiles and the workgroups finish
            // close together.  Indices past the range's real tiles (a last
            // range with fewer groups) hold no tile.
            const int x = (int)(it / p.tper);
            const int64_t local = it - (int64_t)x * p.tper;
            const int64_t r0 = (int64_t)x * p.tgpx;
            const int64_t nrx = max((int64_t)0, min((int64_t)p.tgpx, p.tcum[p.nscenes] - r0));
            const int64_t sx = min((int64_t)p.tranks, nrx);
            const int64_t whole = nrx - sx;
            int64_t grank;
            if (local < whole) {
                grank = r0 + local;
            } else {
                const int64_t j = local - whole;
                if (j >= sx * p.tparts) continue;
                grank = r0 + whole + j / p.tparts;
                part = (int)(j % p.tparts);
            }
            while (sid + 1 < p.nscenes && p.tcum[sid + 1] <= grank) ++sid;
            rank = grank - p.tcum[sid];
        } else {
            while (sid + 1 < p.nscenes && p.tcum[sid + 1] <= it) ++sid;
            const int64_t lt = it - p.tcum[sid];
            const int64_t gpc = ((constant_ptr<SceneDesc>)(p.scenes + sid))->gpc;
            cc = (int)(lt / gpc);
            rank = lt - (int64_t)cc * gpc;
        }
        // The descriptors and tile orders were written by the init kernel and
        // stay fixed during this one: read through the constant address
        // space, so that their uniform fields come in through scalar loads.
        const constant_ptr<SceneDesc> sc = (constant_ptr<SceneDesc>)(p.scenes + sid);
        int t, c0, c1, g;
        {
            if (p.tsplit) {
                c0 = part < 0 ? 0 : part * p.tcpb;
                c1 = part < 0 ? sc->C : min(sc->C, c0 + p.tcpb);
            } else {
                c0 = cc * p.cpb;
                c1 = min(sc->C, c0 + p.cpb);
            }
            const int r = ((constant_ptr<int32_t>)sc->order)[(int)rank];
            t = 0;
            while (t + 1 < sc->T && sc->gcum[t + 1] <= r) ++t;
            g = r - sc->gcum[t];
        }
        const int64_t j0 = (int64_t)g * sc->G;
        const int64_t krem = sc->k[t] - j0;
        const int n = (int)(krem < sc->G ? krem : sc->G);
        const int32_t* J = sc->kept + sc->koff[t] + j0;
        const int nb = sc->nb;
        const int my_bl = tid < nb ? (int)sc->bl[tid] : 0;  // this thread's bit-width (tid < nb)

        // ---- per-element state in registers.  The kept indices and the
        // weights are the same for every channel of the tile: they are
        // gathered once per tile and held, so that a channel costs one
        // round trip (its values).  A group beyond NT * EPT elements (the
        // chunked kernel) is gathered per channel and chunk, again for every
        // histogram batch, its indices and weights from L1/L2.
        constexpr int CAP = NT * EPT;
        const int nchunk = CHUNKED ? (n + CAP - 1) / CAP : 1;
        float u[EPT], xv[EPT], wv[EPT];
        int32_t ids[CHUNKED ? 1 : EPT];

        const float* imp = sc->imp;
        if constexpr (!CHUNKED) {
#pragma unroll
            for (int i = 0; i < EPT; ++i) ids[i] = i * NT + tid < n ? J[i * NT + tid] : 0;
#pragma unroll
            for (int i = 0; i < EPT; ++i) wv[i] = i * NT + tid < n ? imp[ids[i]] : 0.0f;
        }
        // the first batch's bins are cleared before the barrier of the
        // channel's min/max (the later batches clear their own)
        // (t0: an opaque copy of tid, so that the start addresses are made
        // afresh here rather than held, or spilled, across the channel loop;
        // the same below)
        auto clear_batch = [&](int bt) {
            const int words = p.batch_words[bt];
            int t0 = tid;
            asm volatile("" : "+v"(t0));
            uint4* h4 = reinterpret_cast<uint4*>(hist);
            for (int w = t0; w < (words >> 2); w += NT) h4[w] = make_uint4(0u, 0u, 0u, 0u);
            for (int w = (words & ~3) + t0; w < words; w += NT) hist[w] = 0u;
        };
        for (int c = c0; c < c1; ++c) {
            clear_batch(0);
            const float* row = sc->attr + (int64_t)c * sc->ld;
            const int64_t slot = ((int64_t)t * sc->C + c) * sc->gmaxn + g;
            float mn = INFINITY, mx = -INFINITY, wm = 0.0f;  // wm: largest |weight|
            uint32_t bad = 0;
            auto gather = [&](int ch) {
                // Opaque copies of the index and weight pointers: otherwise
                // their loads are hoisted out of the channel loop and held in
                // registers across all channels.
                // (typed global: an opaque generic pointer would make flat loads)
                global_ptr<const int32_t> Jc = (global_ptr<const int32_t>)J;
                global_ptr<const float> impc = (global_ptr<const float>)imp;
                asm volatile("" : "+v"(Jc), "+v"(impc));
                const global_ptr<const float> rowg = (global_ptr<const float>)row;
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    int j = ch * CAP + i * NT + tid;
                    float x = 0.0f, w = 0.0f;
                    if (j < n) {
                        int32_t id = Jc[j];
                        x = rowg[id];
                        w = impc[id];
                        bad |= (uint32_t)(!finite_f32(x) || !finite_f32(w));
                        mn = fminf(mn, x);
                        mx = fmaxf(mx, x);
                        wm = fmaxf(wm, fabsf(w));
                    }
                    xv[i] = x;
                    wv[i] = w;
                }
            };
            if constexpr (CHUNKED) {
                for (int ch = nchunk - 1; ch >= 0; --ch) gather(ch);  // ends holding chunk 0
            } else {
                // every load issued before the first is used: elements past n
                // hold index 0, an in-bounds read of row[0] that is dropped.
                // The opaque copy keeps each index a 32-bit register (a 64-bit
                // offset per element held across channels costs registers).
                const global_ptr<const float> rowg = (global_ptr<const float>)row;
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    int32_t id = ids[i];
                    asm volatile("" : "+v"(id));
                    xv[i] = rowg[id];
                }
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    float x = 0.0f;
                    if (i * NT + tid < n) {
                        x = xv[i];
                        const float w = wv[i];
                        bad |= (uint32_t)(!finite_f32(x) || !finite_f32(w));
                        mn = fminf(mn, x);
                        mx = fmaxf(mx, x);
                        wm = fmaxf(wm, fabsf(w));
                    }
                    xv[i] = x;
                }
            }
            mn = wave_min_dpp(mn);
            mx = wave_max_dpp(mx);
            wm = wave_max_dpp(wm);
            bad = wave_or_dpp(bad);
            if (lane == 0) {
                red_mn[wave] = mn;
                red_mx[wave] = mx;
                red_w[wave] = wm;
                red_bad[wave] = bad;
            }
            __syncthreads();
            mn = red_mn[0];
            mx = red_mx[0];
            wm = red_w[0];
            bad = red_bad[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                mn = fminf(mn, red_mn[w]);
                mx = fmaxf(mx, red_mx[w]);
                wm = fmaxf(wm, red_w[w]);
                bad |= red_bad[w];
            }
            const float R = mx - mn;
            if (!finite_f32(R)) bad = 1;
            if (tid == 0) {
                sc->gmin[slot] = mn;
                sc->gmax[slot] = mx;
            }
            if (bad || R == 0.0f) {
                // non-finite group: NaN tables and the status flag; constant
                // group: every code 0, zero loss and zero size.
                if (tid < nb) {
                    sc->err[slot * nb + tid] = bad ? NAN : 0.0;
                    sc->bits[slot * nb + tid] = bad ? NAN : 0.0;
                    if (!bad && sc->hist) sc->hist[slot * sc->hist_bins + sc->hoff[tid]] = (uint32_t)n;
                }
                if (bad && tid == 0) atomicOr(&p.status->nonfinite, 1u);
                __syncthreads();
                continue;
            }

            // ---- per-b scale and zero point (literal FP32 definition)
            if (tid < nb) {
                float P = ldexpf(1.0f, my_bl);
                float S = R / P;
                float Z = 0.0f;
                if (S != 0.0f) {
                    float r = mx / S;
                    Z = __builtin_rintf(P - r);
                }
                int t0 = tid;
                asm volatile("" : "+v"(t0));
                prmS[t0] = S;
                prmZ[t0] = Z;
            }
            // a range that underflows at some b (S_b = 0; S only shrinks with b)
            const bool anyzero = R / ldexpf(1.0f, sc->bmax) == 0.0f;
            for (int i = tid; i < MGS_MAX_BITS * NW; i += NT) {
                (&bitpart[0][0])[i] = 0.0;
                (&errpart[0][0])[i] = 0.0;
            }
            const bool fast = R >= ldexpf(1.0f, sc->bmax - 126);
            // Fast tiles evaluate the loss on x * 2^-E with 2^E <= R < 2^(E+1)
            // (R is normal here): every step S_b * 2^-E is then normal and near
            // 2^-b, and the terms are rescaled by 2^(2E) in FP64.
            const int E = fast ? (int)((__float_as_uint(R) >> 23) & 0xFFu) - 127 : 0;
            const double esc = ldexp(1.0, 2 * E);
            // u = x / R, correctly rounded, without a division per element:
            // with Rs = R * 2^-E in [1, 2) and y = RN(1 / Rs), q = RN(xs * y)
            // is within 1.5 ulp of xs / Rs; one correction by the exact FMA
            // remainder xs - Rs * q makes it faithful, and a second one the
            // correctly rounded quotient (Markstein's theorem: y within half an
            // ulp of 1 / Rs, q within one ulp of xs / Rs).  The remainders are
            // exact while |xs| >= 2^-100; below that both quotients are under
            // 2^-100 in magnitude, far too small to move fma(u, 2^b, Z) off Z
            // (|Z| >= 1) or, for Z = 0, t + 2^23 off 2^23, so the codes agree.
            const float Rs = ldexpf(R, -E);
            const float yr = fast ? 1.0f / Rs : 0.0f;
            auto quotients = [&]() {
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    const float xs = ldexpf(xv[i], -E);
                    float q = 0.0f;
                    if (fast) {
                        q = xs * yr;
                        float r = __builtin_fmaf(-Rs, q, xs);
                        q = __builtin_fmaf(r, yr, q);
                        r = __builtin_fmaf(-Rs, q, xs);
                        q = __builtin_fmaf(r, yr, q);
                    }
                    u[i] = q;
                    xv[i] = xs;
                    // one element at a time: the next one starts after this
                    // quotient (interleaving them all costs registers)
                    if (i + 1 < EPT) asm volatile("" : "+v"(u[i]), "+v"(xv[i + 1]));
                }
            };
            quotients();
            for (int i = tid; i < p.nbatches; i += NT) ovf_flag[i] = 0u;
            __syncthreads();

            // ---- histogram batches
            for (int bt = 0; bt < p.nbatches; ++bt) {
                const int e0 = p.batch_begin[bt], e1 = p.batch_begin[bt + 1];
                if (bt > 0) {
                    clear_batch(bt);
                    __syncthreads();
                }
                uint32_t ovf = 0;  // some bin grew past the LDS increment table
                for (int ch = 0; ch < nchunk; ++ch) {
                    if constexpr (CHUNKED) {
                        if (nchunk > 1) {
                            gather(ch);
                            quotients();
                        }
                    }
                    const int nc = min(CAP, n - ch * CAP);  // elements of this chunk
                    const bool check = nc < CAP;
                    for (int e = e0; e < e1; ++e) {
                        const HistEntry en = p.entries[e];
                        const int bi = en.bi;
                        const float S = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(prmS[bi])));
                        const float Z = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(prmZ[bi])));
                        const float P = ldexpf(1.0f, en.b);
                        const float Ss = ldexpf(S, -E);
                        const int base = en.lds_off - en.lo;
                        const int rl = en.rlog;
                        const int cpy = lane & ((1 << rl) - 1);
                        Part acc{0.0f, 0.0, 0.0};
                        if (S == 0.0f) {
                            // the range underflows at this b: every code is 0, xhat = min
                            // (all counts go to bin 0: its entropy terms come from the scan)
                            if (en.lo == 0 && tid == 0) hist[en.lds_off] += (uint32_t)nc;
                            if (en.first) {
#pragma unroll
                                for (int i = 0; i < EPT; ++i) {
                                    if (i * NT + tid < nc) {
                                        double d = (double)mn - as_f64(xv[i]);
                                        acc.err64 = __builtin_fma(as_f64(wv[i]), d * d, acc.err64);
                                    }
                                }
                            }
                        } else if (fast && fabsf(Z) <= 8388608.0f && (en.packed || !en.split)) {
                            uint32_t seen = 0;
                            // byte address of bin word w: base + w, in the 0x4B000000-biased
                            // form the fast path uses (see eval_fast)
                            const uint32_t wlo = hist_lds + 4u * (uint32_t)en.lds_off;
                            uint32_t cadj = en.packed
                                                ? hist_lds + 4u * (uint32_t)base - (0x4B000000u << 1)
                                                : hist_lds + 4u * (uint32_t)(base + cpy) - (0x4B000000u << (rl + 2));
                            asm volatile("" : "+v"(cadj));
                            if (en.packed)
                                acc = eval_fast_dispatch<NT, EPT, true>(check, en.rtn, en.split, en.first, cadj, wlo,
                                                                        4u * (uint32_t)en.nwords, 0, u, xv, wv, nc,
                                                                        tid, P, Ss, Z, lf, seen);
                            else
                                acc = eval_fast_dispatch<NT, EPT, false>(check, en.rtn, false, true, cadj, wlo,
                                                                         4u * (uint32_t)en.nwords, rl, u, xv, wv,
                                                                         nc, tid, P, Ss, Z, lf, seen);
                            ovf |= seen & big_count_mask(en.packed);
                        } else {
                            uint32_t seen = 0;
                            acc = eval_generic<NT, EPT>(u, xv, wv, nc, tid, P, S, Ss, Z, hist, base, en.lo,
                                                        en.nwords, en.packed, rl, cpy, !fast, en.first,
                                                        en.rtn, lf, seen);
                            ovf |= seen & big_count_mask(en.packed);
                        }
                        if (en.first) {
                            double tot;
                            if (fast && S != 0.0f) {
                                // FP32 terms (scaled by 2^-2E): trusted when finite and
                                // large enough that underflowed terms cannot matter
                                const float t32 = wave_total_f32(acc.err);
                                if (__builtin_isfinite(t32) && t32 >= (wm + 1.0f) * 0x1p-112f)
                                    tot = (double)t32 * esc;
                                else
                                    tot = wave_total_f64(loss_f64<NT, EPT>(u, xv, wv, nc, tid, P, Ss, Z)) * esc;
                            } else {
                                tot = wave_total_f64(acc.err64);
                            }
                            if (lane == 0) errpart[bi][wave] += tot;
                        }
                        if (en.rtn && S != 0.0f) {
                            const double tot = wave_total_f64(acc.ent);
                            if (lane == 0) bitpart[bi][wave] += tot;
                        }
                    }
                }
                // one barrier: the wavefronts that saw a large count flag the
                // batch before it, everyone reads the flag after it
                if (__builtin_amdgcn_ballot_w64(ovf != 0u) != 0 && lane == 0) atomicOr(&ovf_flag[bt], 1u);
                __syncthreads();
                const bool any_ovf = ovf_flag[bt] != 0u;
                const bool dbg = sc->hist != nullptr;
                // ---- entropy terms of the scanned histograms (the batch's
                // first entries): one lane per bin, which adds up the bin's
                // 2^rlog copies from its adjacent words (16-byte reads); the
                // wavefronts take the bins in 64-bin slices, the first slice
                // of each entry on a wavefront that rotates with the entry, and
                // only wavefronts that held a slice sum their lanes.
                if (!dbg) {
                    for (int e = e0; e < p.batch_scan_end[bt]; ++e) {
                        const HistEntry en = p.entries[e];
                        const int rl = en.rlog, R = 1 << rl;
                        const int nq = en.nwords >> rl;  // bins (packed: words of two bins)
                        const int first_w = (e * 5) % NW;
                        const int slice = wave >= first_w ? wave - first_w : wave + NW - first_w;
                        if (slice * MGS_WAVE >= nq) continue;
                        double s = 0.0;
                        for (int q = slice * MGS_WAVE + lane; q < nq; q += NT) {
                            const uint32_t* src = hist + en.lds_off + (q << rl);
                            uint32_t h = 0;
                            if (R >= 4) {
                                for (int k = 0; k < R; k += 4) {
                                    const uint4 v = *reinterpret_cast<const uint4*>(src + k);
                                    h += (v.x + v.y) + (v.z + v.w);
                                }
                            } else if (R == 2) {
                                const uint2 v = *reinterpret_cast<const uint2*>(src);
                                h = v.x + v.y;
                            } else {
                                h = src[0];
                            }
                            if (en.packed)
                                s += hlog2h(h & 0xFFFFu, lg, lgt) + hlog2h(h >> 16, lg, lgt);
                            else
                                s += hlog2h(h, lg, lgt);
                        }
                        const double tot = wave_total_f64(s);
                        if (lane == 0) bitpart[en.bi][wave] += tot;
                    }
                }
                // ---- the rest: incremental entries whose range underflows at
                // this b (every count in bin 0: scanned), the corrections of
                // incremental ones whose bins outgrew the LDS table (a bin of
                // h > LGTAB got floor(h / LGTAB) full cycles of the increments plus
                // the first h mod LGTAB of them, and needs R(T(h)) on the same
                // grid), and, with the optional debug copy of the bins, every
                // entry (scanned ones included)
                const int e_beg = dbg ? e0 : p.batch_scan_end[bt];
                const int e_end = (any_ovf || anyzero || dbg) ? e1 : p.batch_scan_end[bt];
                for (int e = e_beg; e < e_end; ++e) {
                    const HistEntry en = p.entries[e];
                    const bool scan = !en.rtn || (anyzero && prmS[en.bi] == 0.0f);
                    const bool fix = !scan && any_ovf;
                    uint32_t* hout = sc->hist ? sc->hist + slot * sc->hist_bins + sc->hoff[en.bi] : nullptr;
                    if (!scan && !fix && !hout) continue;
                    double s = 0.0;
                    auto term = [&](uint32_t h) {
                        if (scan) s += hlog2h(h, lg, lgt);
                        else if (fix && h > (uint32_t)LGTAB)
                            s += grid_round(lgt[h], p.kgrid) - (double)(h / LGTAB) * rt_cycle -
                                 grid_round(lg[h % LGTAB], p.kgrid);
                    };
                    if (en.rlog) {
                        // replicated bins: the 2^rlog copies of a bin sit in adjacent
                        // lanes of one wavefront; DPP row shifts sum them into the
                        // group's last lane
                        const int rl = en.rlog, R = 1 << rl;
                        for (int w0 = 0; w0 < en.nwords; w0 += NT) {
                            const int w = w0 + tid;
                            const uint32_t h =
                                group_sum_u32(w < en.nwords ? hist[en.lds_off + w] : 0u, rl);
                            if ((lane & (R - 1)) == R - 1 && w < en.nwords) {
                                term(h);
                                if (hout) hout[en.lo + (w >> rl)] = h;
                            }
                        }
                    } else {
                        for (int w = tid; w < en.nwords; w += NT) {
                            uint32_t v = hist[en.lds_off + w];
                            if (!en.packed) {
                                term(v);
                                if (hout) hout[en.lo + w] = v;
                            } else {
                                uint32_t h0 = v & 0xFFFFu, h1 = v >> 16;
                                term(h0);
                                term(h1);
                                if (hout) {
                                    hout[2 * (en.lo + w)] = h0;
                                    hout[2 * (en.lo + w) + 1] = h1;
                                }
                            }
                        }
                    }
                    if (scan || fix) {
                        const double tot = wave_total_f64(s);
                        if (lane == 0) bitpart[en.bi][wave] += tot;
                    }
                }
                __syncthreads();
            }

            // ---- finalize the tile's table entries
            if (tid < nb) {
                double e = 0.0, s = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    e += errpart[tid][w];
                    s += bitpart[tid][w];
                }
                sc->err[slot * nb + tid] = e;
                sc->bits[slot * nb + tid] = lgt[n] - s;  // n log2 n - sum_k h_k log2 h_k
            }
            __syncthreads();
        }
    }
}

// Copies one scene descriptor (a by-value kernel argument) into device memory.
__global__ void scene_copy_kernel(SceneDesc sd, SceneDesc* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = sd;
}

// Position of group g of a ratio with k kept Gaussians along the Gaussian
// index: the middle of its run of kept positions as a fraction of k,
// (2 g G + n) times inv = 1 / (2 k) (every position is computed the same
// way, so the positions of one ratio increase with g and all of them are
// ordered consistently).  Kept indices ascend, so groups of different ratios
// at similar positions read nearby Gaussians.
__device__ __forceinline__ double group_pos(int64_t k, int G, int g, double inv) {
    const int64_t j0 = (int64_t)g * G;
    const int64_t n = min((int64_t)G, k - j0);
    return (double)(2 * j0 + n) * inv;
}

// Tile order of a channel run: its groups sorted by (position, ratio).  The
// rank of group (t, g) counts, per ratio, the groups before it (positions
// increase with g, so a binary search per ratio); order[rank] = r.  The keep
// counts and group prefixes come from LDS copies (sk, sg): the searches are
// chains of dependent reads.
__device__ void tile_order(const SceneDesc* sc, const int64_t* sk, const int32_t* sg, int r) {
    const int T = sc->T, G = sc->G;
    int t = 0;
    while (t + 1 < T && sg[t + 1] <= r) ++t;
    const int g = r - sg[t];
    const double pos = group_pos(sk[t], G, g, 1.0 / (double)(2 * sk[t]));
    int rank = g;
    for (int u = 0; u < T; ++u) {
        if (u == t) continue;
        const int64_t ku = sk[u];
        const double inv = 1.0 / (double)(2 * ku);
        int lo = 0, hi = sg[u + 1] - sg[u];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const double pm = group_pos(ku, G, mid, inv);
            if (pm < pos || (pm == pos && u < t)) lo = mid + 1;
            else hi = mid;
        }
        rank += lo;
    }
    sc->order[rank] = r;
}

// Empty slots (groups past ceil(k_t / G)) hold NaN; the debug histogram is
// cleared; the status word is reset; every scene gets its tile order.
__global__ void sweep_init_kernel(SceneDesc* __restrict__ scenes, int count,
                                  mgs_status_block* status, double* lgtab, int lgtab_max, int K) {
    if (blockIdx.x == 0 && threadIdx.x < 16) {
        if (threadIdx.x == 0) status->nonfinite = 0u;
        status->queue[threadIdx.x] = 0u;
    }
    // T(h) = h log2 h for every count a group can hold (FP64, 0 for h < 2),
    // and the increments F[c] = R(T(c+1)) - R(T(c)) with R the rounding to the
    // grid 2^-K: sums of increments telescope to R(T(h)) exactly, in any order
    double* inc = lgtab + (lgtab_max + 1);
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h <= lgtab_max; h += gridDim.x * blockDim.x) {
        const double dh = (double)h, dh1 = (double)(h + 1);
        const double t0 = h < 2 ? 0.0 : dh * log2(dh);
        const double t1 = dh1 * log2(dh1);
        lgtab[h] = t0;
        inc[h] = grid_round(t1, K) - grid_round(t0, K);
    }
    __shared__ int64_t sk[MGS_MAX_RATIOS];
    __shared__ int32_t sg[MGS_MAX_RATIOS + 1];
    for (int s = 0; s < count; ++s) {
        SceneDesc* sc = &scenes[s];
        if ((int64_t)blockIdx.x * blockDim.x < sc->gpc) {  // (block-uniform) this block orders groups
            __syncthreads();  // the previous scene's searches are done with sk, sg
            for (int u = threadIdx.x; u <= sc->T; u += blockDim.x) {
                if (u < sc->T) sk[u] = sc->k[u];
                sg[u] = sc->gcum[u];
            }
            __syncthreads();
            for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < sc->gpc; r += gridDim.x * blockDim.x)
                tile_order(sc, sk, sg, r);
        }
        const int64_t nslot = (int64_t)sc->T * sc->C * sc->gmaxn;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslot;
             i += (int64_t)gridDim.x * blockDim.x) {
            int t = (int)(i / ((int64_t)sc->C * sc->gmaxn));
            int g = (int)(i % sc->gmaxn);
            int ng = sc->gcum[t + 1] - sc->gcum[t];
            if (g >= ng) {
                for (int b = 0; b < sc->nb; ++b) {
                    sc->err[i * sc->nb + b] = NAN;
                    sc->bits[i * sc->nb + b] = NAN;
                }
                sc->gmin[i] = NAN;
                sc->gmax[i] = NAN;
            }
            if (sc->hist)
                for (int64_t b = 0; b < sc->hist_bins; ++b) sc->hist[i * sc->hist_bins + b] = 0u;
        }
    }
}

// ------------------------------------------------------------------ host side

template <int NT, int EPT, bool CHUNKED>
static hipError_t launch_one(const SweepParams& p, int64_t grid, size_t lds,
                             hipStream_t s) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)sweep_kernel<NT, EPT, CHUNKED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)e;
    }
    hipLaunchKernelGGL((sweep_kernel<NT, EPT, CHUNKED>), dim3((unsigned)grid), dim3(NT), lds, s, p);
    return hipGetLastError();
}

struct Variant {
    int nt, ept;
    bool chunked;
    hipError_t (*fn)(const SweepParams&, int64_t, size_t, hipStream_t);
    const void* kern;
};

#define MGS_V(NT, EPT) \
    {NT, EPT, false, &launch_one<NT, EPT, false>, (const void*)&sweep_kernel<NT, EPT, false>}
#define MGS_VC(NT, EPT) \
    {NT, EPT, true, &launch_one<NT, EPT, true>, (const void*)&sweep_kernel<NT, EPT, true>}
static const Variant kVariants[] = {
    MGS_V(256, 1),  MGS_V(256, 2),  MGS_V(256, 4),  MGS_V(256, 8),  MGS_V(256, 16), MGS_V(256, 32),
    MGS_V(512, 1),  MGS_V(512, 2),  MGS_V(512, 4),  MGS_V(512, 8),  MGS_V(512, 16), MGS_V(512, 32),
    MGS_V(1024, 1), MGS_V(1024, 2), MGS_V(1024, 4), MGS_V(1024, 8), MGS_V(1024, 16),
    MGS_VC(512, 16),  // groups larger than any register-resident shape
};
#undef MGS_V
#undef MGS_VC

// A non-chunked variant when nt * ept covers the group, else the chunked one.
static const Variant* find_variant(int nt, int ept, int G = 0) {
    const bool need_chunk = (int64_t)nt * ept < G;
    for (const Variant& v : kVariants)
        if (v.nt == nt && v.ept == ept && v.chunked == need_chunk) return &v;
    return nullptr;
}

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
Shape variant_shape(int i) { return Shape{kVariants[i].nt, kVariants[i].ept, 0}; }
bool variant_chunked(int i) { return kVariants[i].chunked; }

static int device_attr(hipDeviceAttribute_t a, int fallback) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fallback;
    if (hipDeviceGetAttribute(&v, a, dev) != hipSuccess || v <= 0) return fallback;
    return v;
}

static int device_lds_bytes() {
    static int cached = 0;
    if (!cached) cached = device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536);
    return cached;
}

int device_cus() {
    static int cached = 0;
    if (!cached) cached = device_attr(hipDeviceAttributeMultiprocessorCount, 256);
    return cached;
}

// Static LDS of a kernel variant (everything but the histogram words), with
// room for the tile index of the persistent grid and the 16-byte alignment
// of the histogram words.
static int static_lds_bytes(int nt) {
    int nw = nt / MGS_WAVE;
    return (int)(2 * sizeof(double) * LGTAB + 2 * sizeof(double) * MGS_MAX_BITS * nw + 4 * 4 * nw +
                 2 * 4 * MGS_MAX_BITS + 4 * MGS_MAX_ENTRIES + sizeof(int64_t)) + 256 + 16;
}

#ifndef MGS_RTN_FACTOR
#define MGS_RTN_FACTOR 0.0625
#endif
// Entropy from the atomics' old counts (incremental) instead of a scan of the
// bins, for bit-widths with more bins than a sixteenth of the group's
// elements.  The increments add work to every pass, where other wavefronts
// hide their latency; a scan runs between barriers, with every wavefront of
// the workgroup waiting on its loads at once (measured crossover).
static bool incremental_entropy(int b, int G) {
    return (double)((int64_t)1 << b) > MGS_RTN_FACTOR * (double)G;
}

// Two 16-bit bins per LDS word: for a bit-width whose bins do not fit one
// batch unpacked, and for incremental ones with at least as many bins as the
// group has elements (counts mostly 0-2; 16 bits hold any group, G <= 65535).
// Packing costs about five VALU operations per evaluation but halves the
// words to clear and lets the plan use fewer or smaller batches (measured:
// 18.4 -> 17.9 ms at G = 16384, b = 1..16).
static bool packed_bins(int b, int G, int cap_words) {
    const int64_t full = (int64_t)1 << b;
    return full > cap_words || (incremental_entropy(b, G) && full >= G);
}

bool build_plan(const uint8_t* bl, int nb, int cap_words, int G, SweepParams* p) {
    // Greedy: largest histograms first, each into the first batch with room;
    // a b larger than a whole batch is split into windows of cap_words.
    // Scanned histograms with few bins get lane-interleaved copies (up to
    // repl_words words) so that lanes landing in one bin do not serialise on
    // one LDS address.  Fixed-size arrays only: planning allocates nothing.
    struct Item { int bi; int words; bool packed; int rlog; };
    if (nb < 1 || nb > MGS_MAX_BITS) return false;
    // whole 16-byte units only: every window and entry starts on a unit
    // boundary (the scans read the copies of a bin as 16-byte units)
    cap_words &= ~3;
    // words the copies of one scanned histogram may take: more for larger
    // groups, whose lanes crowd the same bins more (measured at G = 16384)
    const int repl_words = std::max(REPL_WORDS, G / 8);
    Item items[MGS_MAX_BITS];
    for (int i = 0; i < nb; ++i) {
        int full = 1 << bl[i];
        bool rtn = incremental_entropy(bl[i], G);
        bool packed = packed_bins(bl[i], G, cap_words);
        int rlog = 0;
        if (!packed && !rtn)
            while (rlog < REPL_MAX_LOG && (full << (rlog + 1)) <= std::min(repl_words, cap_words)) ++rlog;
        // insertion keeps equal sizes in list order (a stable sort, largest first)
        Item it{i, packed ? full / 2 : full << rlog, packed, rlog};
        int pos = i;
        while (pos > 0 && items[pos - 1].words < it.words) {
            items[pos] = items[pos - 1];
            --pos;
        }
        items[pos] = it;
    }
    HistEntry bent[MGS_MAX_ENTRIES][MGS_MAX_ENTRIES];
    int bcount[MGS_MAX_ENTRIES], used[MGS_MAX_ENTRIES];
    int nbat = 0, ne = 0;
    for (int ii = 0; ii < nb; ++ii) {
        const Item& it = items[ii];
        if (it.words > cap_words) {
            for (int lo = 0; lo < it.words; lo += cap_words) {
                if (nbat == MGS_MAX_ENTRIES || ne == MGS_MAX_ENTRIES) return false;
                HistEntry e{};
                e.bi = it.bi;
                e.b = bl[it.bi];
                e.packed = it.packed;
                e.first = lo == 0;
                e.split = 1;
                e.rtn = incremental_entropy(bl[it.bi], G);
                e.lo = lo;
                e.nwords = std::min(cap_words, it.words - lo);
                e.lds_off = 0;
                bent[nbat][0] = e;
                bcount[nbat] = 1;
                used[nbat] = (e.nwords + 3) & ~3;
                ++nbat;
                ++ne;
            }
            continue;
        }
        int k = 0;
        for (; k < nbat; ++k)
            if (used[k] + ((it.words + 3) & ~3) <= cap_words) break;
        if (k == nbat) {
            if (nbat == MGS_MAX_ENTRIES) return false;
            bcount[nbat] = 0;
            used[nbat] = 0;
            ++nbat;
        }
        if (ne == MGS_MAX_ENTRIES) return false;
        HistEntry e{};
        e.bi = it.bi;
        e.b = bl[it.bi];
        e.packed = it.packed;
        e.rlog = it.rlog;
        e.first = 1;
        e.split = 0;
        e.rtn = incremental_entropy(bl[it.bi], G);
        e.lo = 0;
        e.nwords = it.words;
        e.lds_off = used[k];
        used[k] += (it.words + 3) & ~3;  // every entry starts 16-byte aligned
        bent[k][bcount[k]++] = e;
        ++ne;
    }
    p->nbatches = nbat;
    p->nentries = ne;
    p->max_batch_words = 0;
    int e = 0;
    for (int k = 0; k < nbat; ++k) {
        p->batch_begin[k] = e;
        p->batch_words[k] = used[k];
        p->max_batch_words = std::max(p->max_batch_words, used[k]);
        // scanned entries first (their order inside a batch changes nothing:
        // each b has at most one window per batch)
        for (int x = 0; x < bcount[k]; ++x)
            if (!bent[k][x].rtn) p->entries[e++] = bent[k][x];
        p->batch_scan_end[k] = e;
        for (int x = 0; x < bcount[k]; ++x)
            if (bent[k][x].rtn) p->entries[e++] = bent[k][x];
    }
    p->batch_begin[nbat] = e;
    return true;
}

int plan_for(const SceneDesc& sc, const Shape& sh, SweepParams* p, size_t* lds_bytes) {
    int devlds = device_lds_bytes();
    int cap = sh.lds_cap > 0 ? std::min(sh.lds_cap, devlds) : devlds;
    int cap_words = (cap - static_lds_bytes(sh.nt)) / 4;
    // keep the capacity a power of two so bin windows tile 2^b evenly
    int pw = 1024;
    while (pw * 2 <= cap_words) pw *= 2;
    if (!build_plan(sc.bl, sc.nb, pw, sc.G, p)) return MGS_EINVAL;
    *lds_bytes = (size_t)p->max_batch_words * 4;
    return MGS_OK;
}

int fill_scene(const mgs_sweep_desc* d, const float* attr, const float* imp, const int32_t* kept,
               double* err, double* bits, float* gmin, float* gmax, uint32_t* hist, SceneDesc* sc) {
    if (!d || !d->h_k || !d->h_bits) return MGS_EINVAL;
    if (d->C < 1 || d->T < 1 || d->T > MGS_MAX_RATIOS || d->G < 1 || d->G > MGS_MAX_GROUP ||
        d->nb < 1 || d->nb > MGS_MAX_BITS || d->N < 0 || d->N >= ((int64_t)1 << 31) || d->ld < d->N)
        return MGS_EINVAL;
    for (int i = 0; i < d->nb; ++i) {
        if (d->h_bits[i] < 1 || d->h_bits[i] > MGS_MAX_BITS) return MGS_EINVAL;
        if (i && d->h_bits[i] <= d->h_bits[i - 1]) return MGS_EINVAL;
    }
    std::memset(sc, 0, sizeof(*sc));
    int64_t kmax = 0, off = 0;
    int64_t gc = 0;
    for (int t = 0; t < d->T; ++t) {
        int64_t k = d->h_k[t];
        if (k < 0 || k > d->N) return MGS_EINVAL;
        sc->k[t] = k;
        sc->koff[t] = off;
        off += k;
        kmax = std::max(kmax, k);
        sc->gcum[t] = (int32_t)gc;
        gc += (k + d->G - 1) / d->G;
    }
    if (gc >= ((int64_t)1 << 31) / d->C) return MGS_EINVAL;
    sc->gcum[d->T] = (int32_t)gc;
    if (off > 0 && (!kept || !imp || !attr)) return MGS_EINVAL;
    if (!err || !bits || !gmin || !gmax) return MGS_EINVAL;
    sc->attr = attr;
    sc->imp = imp;
    sc->kept = kept;
    sc->err = err;
    sc->bits = bits;
    sc->gmin = gmin;
    sc->gmax = gmax;
    sc->hist = hist;
    sc->ld = d->ld;
    sc->C = d->C;
    sc->T = d->T;
    sc->G = d->G;
    sc->nb = d->nb;
    sc->gmaxn = (int32_t)((kmax + d->G - 1) / d->G);
    sc->gpc = (int32_t)gc;
    sc->bmax = d->h_bits[d->nb - 1];
    int64_t hb = 0;
    for (int i = 0; i < d->nb; ++i) {
        sc->bl[i] = d->h_bits[i];
        sc->hoff[i] = hb;
        hb += (int64_t)1 << d->h_bits[i];
    }
    sc->hist_bins = hb;
    return MGS_OK;
}

bool shape_valid(const Shape& sh, int G) { return find_variant(sh.nt, sh.ept, G) != nullptr; }

// Default launch shape: the fewest elements per thread that still gives each
// thread >= 8 of them (or the largest workgroup when G is small); groups
// beyond 1024 x 16 elements are processed in chunks of that size.
Shape default_shape(int G, int nb, int bmax) {
    (void)nb;
    (void)bmax;
    for (int e : {8, 16, 4, 2, 1, 32}) {
        for (int t : {256, 512, 1024}) {
            if ((int64_t)t * e >= G && find_variant(t, e, G)) return Shape{t, e, 0};
        }
    }
    return Shape{512, 16, 0};  // chunked
}

int launch_sweep(const SweepParams& p, const Shape& sh, size_t lds,
                 int64_t grid, hipStream_t s, int G) {
    const Variant* v = find_variant(sh.nt, sh.ept, G);
    if (!v) return MGS_EINVAL;
    // one workgroup per tile, rounded up to whole XCD rounds (the extra
    // workgroups find no tile); a persistent grid fills every resident slot
    // of the device (whole XCD rounds), but never exceeds that first grid
    const int64_t per_tile = (p.ntiles + MGS_XCDS - 1) / MGS_XCDS * MGS_XCDS;
    if (p.persist) {
        const int64_t slots = (int64_t)max_resident_blocks(sh, lds, G) * device_cus();
        grid = std::min(per_tile, std::max<int64_t>(MGS_XCDS, slots / MGS_XCDS * MGS_XCDS));
    } else if (grid <= 0 || grid > p.ntiles) {
        grid = per_tile;
    }
    if (p.ntiles < 1) return MGS_OK;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    return v->fn(p, grid, lds, s) == hipSuccess ? MGS_OK : MGS_EDEVICE;
}

int launch_init(const SceneDesc* host_scenes, int count, SceneDesc* d_scenes,
                mgs_status_block* status, double* lgtab, int lgtab_max, hipStream_t s) {
    int64_t slots = 0;
    for (int i = 0; i < count; ++i) {
        hipLaunchKernelGGL(scene_copy_kernel, dim3(1), dim3(64), 0, s, host_scenes[i], d_scenes + i);
        slots = std::max(slots, (int64_t)host_scenes[i].T * host_scenes[i].C * host_scenes[i].gmaxn);
    }
    int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((slots + 255) / 256, 2048));
    blocks = std::max<int64_t>(blocks, (lgtab_max + 256) / 256);
    blocks = std::min<int64_t>(blocks, 2048);
    hipLaunchKernelGGL(sweep_init_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_scenes, count,
                       status, lgtab, lgtab_max, increment_grid_bits(lgtab_max));
    return mgs_last_launch();
}

int increment_grid_bits(int G) {
    // largest total: sum over <= G elements of increments <= (G log2 G + G)
    const double top = (double)G * std::log2((double)std::max(G, 2)) + (double)G + 1.0;
    int bits = (int)std::ceil(std::log2(top));
    return 52 - bits;
}

int max_resident_blocks(const Shape& sh, size_t lds, int G) {
    const Variant* v = find_variant(sh.nt, sh.ept, G);
    if (!v) return 1;
    if (lds > 65536) (void)hipFuncSetAttribute(v->kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int nblk = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, v->kern, sh.nt, lds) != hipSuccess ||
        nblk < 1)
        nblk = 1;
    return nblk;
}

// ------------------------------------------------------------------ autotune registry

namespace {
struct TunedEntry { int G, nb, bmax; Shape sh; };
std::mutex g_tune_mu;
std::vector<TunedEntry> g_tuned;
}  // namespace

bool tuned_shape(int G, int nb, int bmax, Shape* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TunedEntry& e : g_tuned)
        if (e.G == G && e.nb == nb && e.bmax == bmax) {
            *out = e.sh;
            return true;
        }
    return false;
}

void set_tuned_shape(int G, int nb, int bmax, const Shape& sh) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TunedEntry& e : g_tuned)
        if (e.G == G && e.nb == nb && e.bmax == bmax) {
            e.sh = sh;
            return;
        }
    g_tuned.push_back({G, nb, bmax, sh});
}

}  // namespace mgs

// ------------------------------------------------------------------ C ABI

// Workspace: status word | scene descriptors | h log2 h table [0, G] |
// entropy increments [0, G] | each scene's tile order (one int per group of
// a channel run).
static size_t sweep_ws_scene_off() { return MGS_STATUS_BYTES; }
static size_t sweep_ws_table_off(int nscenes) {
    return sweep_ws_scene_off() + mgs_align_up(sizeof(mgs::SceneDesc) * (size_t)nscenes, 256);
}
static int sweep_ws_clamp_g(int G) { return (G < 1 || G > MGS_MAX_GROUP) ? MGS_MAX_GROUP : G; }
static size_t sweep_ws_order_off(int nscenes, int G) {
    return sweep_ws_table_off(nscenes) +
           mgs_align_up(2 * sizeof(double) * ((size_t)sweep_ws_clamp_g(G) + 1), 256);
}
static size_t sweep_ws_bytes(int nscenes, int G, int64_t groups) {
    return sweep_ws_order_off(nscenes, G) + mgs_align_up(sizeof(int32_t) * (size_t)groups, 256);
}

// Groups per channel run of a descriptor: sum_t ceil(k_t / G), or the bound
// T * ceil(N / G) when the counts are not given.
static int64_t sweep_desc_groups(const mgs_sweep_desc* d) {
    if (!d || d->G < 1 || d->T < 1) return 0;
    const int T = std::min<int>(d->T, MGS_MAX_RATIOS);
    int64_t gc = 0;
    if (d->h_k) {
        for (int t = 0; t < T; ++t) gc += (std::max<int64_t>(d->h_k[t], 0) + d->G - 1) / d->G;
    } else {
        gc = (int64_t)T * ((std::max<int64_t>(d->N, 0) + d->G - 1) / d->G);
    }
    return gc;
}

extern "C" size_t mgs_quant_sweep_ws_bytes(const mgs_sweep_desc* desc) {
    return sweep_ws_bytes(1, desc ? desc->G : MGS_MAX_GROUP, sweep_desc_groups(desc));
}

extern "C" size_t mgs_quant_sweep_multi_ws_bytes(const mgs_sweep_job* h_jobs, int32_t njobs) {
    if (!h_jobs || njobs < 1 || njobs > MGS_MAX_JOBS) return sweep_ws_bytes(MGS_MAX_JOBS, MGS_MAX_GROUP, 0);
    int64_t groups = 0;
    for (int i = 0; i < njobs; ++i) groups += sweep_desc_groups(&h_jobs[i].desc);
    return sweep_ws_bytes(njobs, h_jobs[0].desc.G, groups);
}

// Split tail of a persistent launch: groups cut at the end of each XCD's
// range, and about how many channel runs each.
static constexpr int64_t kTailRanks = 32;
static constexpr int kTailParts = 5;

// One launch over the tiles of `n` scenes that share G and the bit list.
static int sweep_launch_scenes(mgs::SceneDesc* scs, int n, void* d_ws, size_t ws_bytes,
                               hipStream_t s, const mgs::Shape* force) {
    using namespace mgs;
    if (n < 1 || n > MGS_MAX_JOBS) return MGS_EINVAL;
    const SceneDesc& s0 = scs[0];
    for (int i = 1; i < n; ++i) {
        if (scs[i].G != s0.G || scs[i].nb != s0.nb) return MGS_EINVAL;
        for (int b = 0; b < s0.nb; ++b)
            if (scs[i].bl[b] != s0.bl[b]) return MGS_EINVAL;
    }
    int64_t groups = 0;
    for (int i = 0; i < n; ++i) groups += scs[i].gpc;
    if (!d_ws || ws_bytes < sweep_ws_bytes(n, s0.G, groups)) return MGS_EWORKSPACE;
    {  // each scene's tile order in the workspace
        int32_t* ord = (int32_t*)((char*)d_ws + sweep_ws_order_off(n, s0.G));
        for (int i = 0; i < n; ++i) {
            scs[i].order = ord;
            ord += scs[i].gpc;
        }
    }
    Shape sh;
    if (force) {
        sh = *force;
    } else if (!tuned_shape(s0.G, s0.nb, s0.bmax, &sh) || !shape_valid(sh, s0.G)) {
        sh = default_shape(s0.G, s0.nb, s0.bmax);
    }
    if (!shape_valid(sh, s0.G)) return MGS_EINVAL;
    SweepParams p;
    std::memset(&p, 0, sizeof(p));
    size_t lds = 0;
    int rc = plan_for(s0, sh, &p, &lds);
    if (rc) return rc;
    int cmax = 1;
    for (int i = 0; i < n; ++i) cmax = std::max(cmax, (int)scs[i].C);
    p.cpb = sh.cpb > 0 ? sh.cpb : cmax;
    p.nscenes = n;
    p.tcum[0] = 0;
    for (int i = 0; i < n; ++i)
        p.tcum[i + 1] = p.tcum[i] + (int64_t)((scs[i].C + p.cpb - 1) / p.cpb) * scs[i].gpc;
    p.ntiles = p.tcum[n];
    // A persistent launch with all channels per tile (scenes with equal
    // channel counts) ends each XCD's range of groups with the last
    // kTailRanks groups cut into channel runs (about kTailParts of them):
    // whole-group tiles are long, and the workgroups that take the last ones
    // would otherwise finish up to one such tile after the others.
    p.tsplit = 0;
    bool same_c = true;
    for (int i = 1; i < n; ++i) same_c = same_c && scs[i].C == s0.C;
    if (sh.persist && same_c && p.cpb >= s0.C && s0.C >= 2 && groups > 0) {
        const int C = s0.C;
        const int tcpb = (C + kTailParts - 1) / kTailParts;
        const int parts = (C + tcpb - 1) / tcpb;
        if (parts >= 2) {
            const int64_t gpx = (groups + MGS_XCDS - 1) / MGS_XCDS;
            const int64_t ranks = std::min<int64_t>(gpx, kTailRanks);
            p.tsplit = 1;
            p.tcpb = tcpb;
            p.tparts = parts;
            p.tgpx = gpx;
            p.tranks = ranks;
            p.tper = (gpx - ranks) + ranks * parts;
            for (int i = 0; i < n; ++i) p.tcum[i + 1] = p.tcum[i] + scs[i].gpc;  // (groups, not tiles)
            p.ntiles = p.tper * MGS_XCDS;
        }
    }
    auto* status = (mgs_status_block*)d_ws;
    auto* d_sc = (SceneDesc*)((char*)d_ws + sweep_ws_scene_off());
    auto* lgtab = (double*)((char*)d_ws + sweep_ws_table_off(n));
    rc = launch_init(scs, n, d_sc, status, lgtab, s0.G, s);
    if (rc) return rc;
    p.status = status;
    p.scenes = d_sc;
    p.lgtab = lgtab;
    p.lgtab_max = s0.G;
    p.kgrid = increment_grid_bits(s0.G);
    p.persist = sh.persist;
    if (p.ntiles == 0) return MGS_OK;
    return launch_sweep(p, sh, lds, 0, s, s0.G);
}

static int sweep_launch(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                        const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                        float* d_gmax, uint32_t* d_hist, void* d_ws, size_t ws_bytes,
                        hipStream_t s, const mgs::Shape* force) {
    mgs::SceneDesc sc;
    int rc = mgs::fill_scene(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, d_hist, &sc);
    if (rc) return rc;
    return sweep_launch_scenes(&sc, 1, d_ws, ws_bytes, s, force);
}

extern "C" int mgs_quant_sweep(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                               const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                               float* d_gmax, uint32_t* d_hist, void* d_ws, size_t ws_bytes,
                               void* stream) {
    return sweep_launch(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, d_hist, d_ws,
                        ws_bytes, (hipStream_t)stream, nullptr);
}

// ------------------------------------------------------------------ allocation-free form
//
// mgs_quant_sweep_static: the same launch as mgs_quant_sweep with the
// workspace in a file-scope device array, for callers that cannot allocate.
// Host code never passes the array's name to a kernel or a copy (on the host
// it only stands for the symbol): the device address of each GPU's copy is
// taken once per device with hipGetSymbolAddress and kept below.

static __device__ __align__(256) unsigned char scratch[MGS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device (null until taken)
}  // namespace

// Device address of the current device's scratch array.
static int static_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MGS_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MGS_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MGS_OK;
}

extern "C" int mgs_quant_sweep_static(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                                      const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                                      float* d_gmax, uint32_t* d_hist, void* stream) {
    mgs::SceneDesc sc;
    int rc = mgs::fill_scene(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, d_hist, &sc);
    if (rc) return rc;
    // the workspace this launch needs must fit in the array (checked before any HIP call)
    if (sweep_ws_bytes(1, sc.G, sc.gpc) > (size_t)MGS_STATIC_SCRATCH_BYTES) return MGS_EWORKSPACE;
    void* ws = nullptr;
    rc = static_scratch(&ws);
    if (rc) return rc;
    return sweep_launch_scenes(&sc, 1, ws, (size_t)MGS_STATIC_SCRATCH_BYTES, (hipStream_t)stream, nullptr);
}

extern "C" int mgs_quant_sweep_static_status(void* stream) {
    void* ws = nullptr;
    int rc = static_scratch(&ws);
    if (rc) return rc;
    return mgs_status_fetch(ws, stream);
}

extern "C" int mgs_quant_sweep_multi(const mgs_sweep_job* h_jobs, int32_t njobs, void* d_ws,
                                     size_t ws_bytes, void* stream) {
    if (!h_jobs || njobs < 1 || njobs > MGS_MAX_JOBS) return MGS_EINVAL;
    std::vector<mgs::SceneDesc> scs((size_t)njobs);
    for (int i = 0; i < njobs; ++i) {
        const mgs_sweep_job& j = h_jobs[i];
        int rc = mgs::fill_scene(&j.desc, j.d_attr, j.d_imp, j.d_kept, j.d_err, j.d_bits, j.d_gmin,
                                 j.d_gmax, j.d_hist, &scs[(size_t)i]);
        if (rc) return rc;
    }
    return sweep_launch_scenes(scs.data(), njobs, d_ws, ws_bytes, (hipStream_t)stream, nullptr);
}

// Candidate shapes of the autotuner: kernel variants x LDS capacities x
// channels per tile.
static const int kLdsCaps[] = {0, 98304, 65536};
static const int kCpbs[] = {0, 4, 2, 1};
static constexpr int kNumCaps = (int)(sizeof(kLdsCaps) / sizeof(kLdsCaps[0]));
static constexpr int kNumCpbs = (int)(sizeof(kCpbs) / sizeof(kCpbs[0]));

static constexpr int kShapesPerVariant = kNumCaps * kNumCpbs * 2;  // x {tile grid, persistent}

extern "C" int mgs_sweep_shape_count(void) { return mgs::variant_count() * kShapesPerVariant; }

static int candidate_variant(int i) { return i / kShapesPerVariant; }

static mgs::Shape candidate_shape(int i) {
    mgs::Shape sh = mgs::variant_shape(candidate_variant(i));
    const int r = i % kShapesPerVariant;
    sh.lds_cap = kLdsCaps[(r / (kNumCpbs * 2)) % kNumCaps];
    sh.cpb = kCpbs[(r / 2) % kNumCpbs];
    sh.persist = r % 2;
    return sh;
}

extern "C" int mgs_sweep_set_shape(int32_t G, int32_t nb, int32_t bmax, int32_t nt, int32_t ept,
                                   int32_t lds_cap, int32_t cpb, int32_t persist) {
    if (G < 1 || G > MGS_MAX_GROUP || nb < 1 || nb > MGS_MAX_BITS || bmax < 1 || bmax > MGS_MAX_BITS ||
        cpb < 0 || persist < 0 || persist > 1)
        return MGS_EINVAL;
    mgs::Shape sh{nt, ept, lds_cap < 0 ? 0 : lds_cap, cpb, persist};
    if (nt != 0 && !mgs::shape_valid(sh, G)) return MGS_EINVAL;
    mgs::set_tuned_shape(G, nb, bmax, sh);  // nt == 0 clears (falls back to the default)
    return MGS_OK;
}

extern "C" int mgs_sweep_autotune(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                                  const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                                  float* d_gmax, void* d_ws, size_t ws_bytes, void* stream, int32_t reps,
                                  float* h_ms, int32_t* h_shapes, int32_t* h_best) {
    using namespace mgs;
    SceneDesc sc;
    int rc = fill_scene(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, nullptr, &sc);
    if (rc) return rc;
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return MGS_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return MGS_EDEVICE;
    }
    const int n = mgs_sweep_shape_count();
    int status = MGS_OK;
    // every candidate's time (-1: does not apply), kept for the near-tie rule
    float times[1024];
    if (n > 1024) return MGS_EINVAL;
    for (int i = 0; i < n; ++i) times[i] = -1.0f;
    for (int i = 0; i < n && status == MGS_OK; ++i) {
        Shape sh = candidate_shape(i);
        if (h_shapes) {
            h_shapes[5 * i] = sh.nt;
            h_shapes[5 * i + 1] = sh.ept;
            h_shapes[5 * i + 2] = sh.lds_cap;
            h_shapes[5 * i + 3] = sh.cpb;
            h_shapes[5 * i + 4] = sh.persist;
        }
        if (h_ms) h_ms[i] = -1.0f;
        const int64_t capacity = (int64_t)sh.nt * sh.ept;
        const bool chunked = variant_chunked(candidate_variant(i));
        if (chunked != (capacity < sc.G)) continue;
        if (!chunked && capacity >= 4 * (int64_t)std::max(sc.G, 256)) continue;  // mostly idle lanes
        if (!shape_valid(sh, sc.G)) continue;
        rc = sweep_launch(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, nullptr, d_ws,
                          ws_bytes, s, &sh);  // warm-up (and plan check)
        if (rc == MGS_EINVAL) continue;       // plan does not fit this capacity
        if (rc) {
            status = rc;
            break;
        }
        float tmin = 0.0f;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) status = MGS_EDEVICE;
            rc = sweep_launch(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, nullptr, d_ws,
                              ws_bytes, s, &sh);
            if (rc) status = rc;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                status = MGS_EDEVICE;
            float ms = 0.0f;
            if (status == MGS_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) status = MGS_EDEVICE;
            if (status) break;
            tmin = r == 0 ? ms : std::min(tmin, ms);
        }
        if (status) break;
        if (h_ms) h_ms[i] = tmin;
        times[i] = tmin;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status) return status;
    // the fastest shape, except that among shapes within 3 % of it the one
    // with more channels per tile (fewer tiles, so fewer fetches of the
    // tiles' indices and weights) wins; then the faster one
    float best_ms = -1.0f;
    for (int i = 0; i < n; ++i)
        if (times[i] >= 0.0f && (best_ms < 0.0f || times[i] < best_ms)) best_ms = times[i];
    if (best_ms < 0.0f) return MGS_EINVAL;
    auto chans = [&](const Shape& sh) { return sh.cpb > 0 ? std::min(sh.cpb, sc.C) : sc.C; };
    int bi = -1;
    for (int i = 0; i < n; ++i) {
        if (times[i] < 0.0f || times[i] > 1.03f * best_ms) continue;
        if (bi < 0) {
            bi = i;
            continue;
        }
        const int ci = chans(candidate_shape(i)), cb = chans(candidate_shape(bi));
        if (ci > cb || (ci == cb && times[i] < times[bi])) bi = i;
    }
    const Shape best = candidate_shape(bi);
    set_tuned_shape(sc.G, sc.nb, sc.bmax, best);
    if (h_best) {
        h_best[0] = best.nt;
        h_best[1] = best.ept;
        h_best[2] = best.lds_cap;
        h_best[3] = best.cpb;
        h_best[4] = best.persist;
    }
    // leave the tables as the chosen shape computes them
    return sweep_launch(desc, d_attr, d_imp, d_kept, d_err, d_bits, d_gmin, d_gmax, nullptr, d_ws,
                        ws_bytes, s, &best);
}
