/*
 * CPU oracle for the MesonGS++ group-wise quantization sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the HIP path.
 *
 * Plain, slow, obviously correct: every quantity is computed by its
 * definition, in the order the definition states, with FP32 arithmetic where
 * the quantizer is defined on FP32 attributes and FP64 accumulation for the
 * error and size tables.  Build: gcc -O2 -ffp-contract=off (no fast-math, no
 * flush-to-zero), optionally -fopenmp for the independent (tau, channel,
 * group) tiles.
 *
 * Readings of the paper used here (all listed in the design notes):
 *   - rounding is round-half-to-even (rintf under the default rounding mode),
 *     for both the code and the zero point;
 *   - clamp is applied before rounding, exactly as the quantizer equation
 *     writes it;
 *   - the dequantized value is (q - Z) * S in FP32, with S and Z recomputed
 *     from the stored group minimum and maximum;
 *   - a group whose scale S = (max - min) / 2^b is zero (constant group, or a
 *     range so small that S underflows) gets code 0 and value min;
 *   - the loss table is the importance-weighted sum of squared errors;
 *   - the size table is the Shannon bound n * H in bits of the group's codes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENONFINITE (-2)
#define ORC_EINFEASIBLE (-3)
#define ORC_ENOMEM (-4)

/* ------------------------------------------------------------------------ */
/* Reserve-ratio pruning (section "Gaussians Pruning"): keep the k most     */
/* important Gaussians, cutting the least important ones.  Order: larger    */
/* importance first; equal importance -> smaller index first.  Output of    */
/* each ratio in ascending index order, ratios concatenated.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    float v;
    int64_t i;
} orc_pair;

static int orc_cmp_pair(const void* pa, const void* pb) {
    const orc_pair* a = (const orc_pair*)pa;
    const orc_pair* b = (const orc_pair*)pb;
    if (a->v > b->v) return -1;
    if (a->v < b->v) return 1;
    if (a->i < b->i) return -1;
    if (a->i > b->i) return 1;
    return 0;
}

int orc_prune_select(const float* imp, int64_t n, const int64_t* k, int32_t T, int32_t* kept) {
    if (n < 0 || T < 0 || (n > 0 && !imp)) return ORC_EINVAL;
    for (int32_t t = 0; t < T; ++t)
        if (k[t] < 0 || k[t] > n) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(imp[i])) return ORC_ENONFINITE;
    orc_pair* order = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
    int64_t* rank = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!order || !rank) { free(order); free(rank); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) { order[i].v = imp[i]; order[i].i = i; }
    qsort(order, (size_t)n, sizeof(orc_pair), orc_cmp_pair);
    for (int64_t r = 0; r < n; ++r) rank[order[r].i] = r;
    int64_t off = 0;
    for (int32_t t = 0; t < T; ++t) {
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i)
            if (rank[i] < k[t]) kept[off + m++] = (int32_t)i;
        off += m;
    }
    free(order);
    free(rank);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Group-wise asymmetric min-max quantizer (section "Group-wise Attribute   */
/* Quantization"):                                                           */
/*   S = (max - min) / 2^b,  Z = round(2^b - max / S),                       */
/*   q = round(clamp(x / S + Z, 0, 2^b - 1)),                                */
/* and the dequantized value (q - Z) * S.  All operations single FP32 ops.   */
/* ------------------------------------------------------------------------ */
static void orc_group_params(float mn, float mx, int b, float* S_out, float* Z_out) {
    float p2 = ldexpf(1.0f, b);
    float R = mx - mn;
    float S = R / p2;
    float Z = 0.0f;
    if (S != 0.0f) {
        float r = mx / S;
        float y = p2 - r;
        Z = rintf(y);
    }
    *S_out = S;
    *Z_out = Z;
}

static uint16_t orc_code(float x, int b, float S, float Z) {
    if (S == 0.0f) return 0;
    float qmax = ldexpf(1.0f, b) - 1.0f;
    float t = x / S;
    t = t + Z;
    if (t < 0.0f) t = 0.0f;
    if (t > qmax) t = qmax;
    float q = rintf(t);
    return (uint16_t)q;
}

static float orc_value(uint16_t q, float mn, float S, float Z) {
    if (S == 0.0f) return mn;
    float d = (float)q - Z;
    return d * S;
}

/* Size of one group's codes in bits: n * H = sum_k h_k * log2(n / h_k). */
static double orc_entropy_bits(const uint32_t* h, int64_t nbins, int64_t n) {
    double s = 0.0;
    for (int64_t k = 0; k < nbins; ++k) {
        if (h[k] == 0) continue;
        double ratio = (double)n / (double)h[k];
        s += (double)h[k] * log2(ratio);
    }
    return s;
}

/* Bit-width lists: strictly increasing values in [1, 16]. */
static int orc_check_bits(const uint8_t* bl, int32_t nb) {
    if (nb < 1 || nb > 16 || !bl) return 0;
    for (int32_t i = 0; i < nb; ++i) {
        if (bl[i] < 1 || bl[i] > 16) return 0;
        if (i > 0 && bl[i] <= bl[i - 1]) return 0;
    }
    return 1;
}

int64_t orc_hist_bins(const uint8_t* bl, int32_t nb) {
    int64_t s = 0;
    for (int32_t i = 0; i < nb; ++i) s += (int64_t)1 << bl[i];
    return s;
}

/*
 * The loss and size tables of the search (section "Acceleration" and
 * section "Size Estimator"): for each reserve ratio t, channel c and group g
 * of G consecutive kept Gaussians, and each candidate bit-width b,
 *   err[t][c][g][b]  = sum_j w_j * (xhat_j - x_j)^2      (FP64)
 *   bits[t][c][g][b] = sum_k h_k * log2(n / h_k)          (FP64)
 * plus the group minimum / maximum.  Slots of groups beyond ceil(k_t / G)
 * hold NaN.  hist (optional) receives the code histograms, per group the
 * 2^b bins of each b in list order.
 */
int orc_quant_sweep(const float* attr, int64_t ld, int32_t C, int64_t N, const float* imp,
                    const int32_t* kept, const int64_t* k, int32_t T, int32_t G,
                    const uint8_t* bl, int32_t nb, double* err, double* bits,
                    float* gmin, float* gmax, uint32_t* hist) {
    if (C < 1 || T < 1 || G < 1 || G > 65535 || ld < N || N < 0) return ORC_EINVAL;
    if (!orc_check_bits(bl, nb)) return ORC_EINVAL;
    int64_t kmax = 0, ksum = 0;
    for (int32_t t = 0; t < T; ++t) {
        if (k[t] < 0 || k[t] > N) return ORC_EINVAL;
        if (k[t] > kmax) kmax = k[t];
        ksum += k[t];
    }
    for (int64_t j = 0; j < ksum; ++j)
        if (kept[j] < 0 || kept[j] >= N) return ORC_EINVAL;
    int64_t gmaxn = (kmax + G - 1) / G;
    int64_t hbins = orc_hist_bins(bl, nb);
    int64_t* koff = (int64_t*)malloc(sizeof(int64_t) * (size_t)T);
    if (!koff) return ORC_ENOMEM;
    koff[0] = 0;
    for (int32_t t = 1; t < T; ++t) koff[t] = koff[t - 1] + k[t - 1];

    int64_t ntile = (int64_t)T * C * gmaxn;
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t tile = 0; tile < ntile; ++tile) {
        int32_t t = (int32_t)(tile / ((int64_t)C * gmaxn));
        int32_t c = (int32_t)((tile / gmaxn) % C);
        int64_t g = tile % gmaxn;
        int64_t tabo = tile * nb;
        int64_t j0 = g * G;
        int64_t j1 = j0 + G < k[t] ? j0 + G : k[t];
        if (hist) memset(hist + tile * hbins, 0, sizeof(uint32_t) * (size_t)hbins);
        if (j0 >= j1) {
            for (int32_t bi = 0; bi < nb; ++bi) { err[tabo + bi] = NAN; bits[tabo + bi] = NAN; }
            gmin[tile] = NAN;
            gmax[tile] = NAN;
            continue;
        }
        int64_t n = j1 - j0;
        const int32_t* J = kept + koff[t] + j0;
        const float* row = attr + (int64_t)c * ld;
        /* minimum and maximum of the group */
        float mn = row[J[0]], mx = row[J[0]];
        int bad = 0;
        for (int64_t j = 0; j < n; ++j) {
            float x = row[J[j]];
            if (!isfinite(x) || !isfinite(imp[J[j]])) bad = 1;
            if (x < mn) mn = x;
            if (x > mx) mx = x;
        }
        if (!isfinite(mx - mn)) bad = 1;
        gmin[tile] = mn;
        gmax[tile] = mx;
        if (bad) {
#pragma omp atomic write
            status = ORC_ENONFINITE;
            for (int32_t bi = 0; bi < nb; ++bi) { err[tabo + bi] = NAN; bits[tabo + bi] = NAN; }
            continue;
        }
        uint32_t* hl = (uint32_t*)calloc((size_t)65536, sizeof(uint32_t));
        int64_t hoff = 0;
        for (int32_t bi = 0; bi < nb; ++bi) {
            int b = bl[bi];
            int64_t nbins = (int64_t)1 << b;
            float S, Z;
            orc_group_params(mn, mx, b, &S, &Z);
            memset(hl, 0, sizeof(uint32_t) * (size_t)nbins);
            double e_sum = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                float x = row[J[j]];
                uint16_t q = orc_code(x, b, S, Z);
                float xh = orc_value(q, mn, S, Z);
                hl[q] += 1;
                double d = (double)xh - (double)x;
                double e = (double)imp[J[j]] * (d * d);
                e_sum += e;
            }
            err[tabo + bi] = e_sum;
            bits[tabo + bi] = orc_entropy_bits(hl, nbins, n);
            if (hist) memcpy(hist + tile * hbins + hoff, hl, sizeof(uint32_t) * (size_t)nbins);
            hoff += nbins;
        }
        free(hl);
    }
    free(koff);
    return status;
}

/*
 * Final quantization at a chosen allocation: codes[c][j] for the k kept
 * Gaussians of one reserve ratio, group g = j / G with bit-width
 * bits[c][g]; gmin / gmax receive the stored per-group metadata.
 */
int orc_quantize(const float* attr, int64_t ld, int32_t C, int64_t N, const int32_t* kept,
                 int64_t k, int32_t G, const uint8_t* bw, uint16_t* codes, float* gmin,
                 float* gmax) {
    if (C < 1 || G < 1 || G > 65535 || k < 0 || k > N || ld < N) return ORC_EINVAL;
    int64_t ng = (k + G - 1) / G;
    for (int64_t i = 0; i < (int64_t)C * ng; ++i)
        if (bw[i] < 1 || bw[i] > 16) return ORC_EINVAL;
    int status = ORC_OK;
    for (int32_t c = 0; c < C; ++c) {
        const float* row = attr + (int64_t)c * ld;
        for (int64_t g = 0; g < ng; ++g) {
            int64_t j0 = g * G, j1 = j0 + G < k ? j0 + G : k;
            float mn = row[kept[j0]], mx = row[kept[j0]];
            for (int64_t j = j0; j < j1; ++j) {
                float x = row[kept[j]];
                if (!isfinite(x)) status = ORC_ENONFINITE;
                if (x < mn) mn = x;
                if (x > mx) mx = x;
            }
            if (!isfinite(mx - mn)) status = ORC_ENONFINITE;
            gmin[(int64_t)c * ng + g] = mn;
            gmax[(int64_t)c * ng + g] = mx;
            int b = bw[(int64_t)c * ng + g];
            float S, Z;
            orc_group_params(mn, mx, b, &S, &Z);
            for (int64_t j = j0; j < j1; ++j) codes[(int64_t)c * k + j] = orc_code(row[kept[j]], b, S, Z);
        }
    }
    return status;
}

int orc_dequantize(const uint16_t* codes, int64_t k, int32_t C, int32_t G, const uint8_t* bw,
                   const float* gmin, const float* gmax, float* out) {
    if (C < 1 || G < 1 || G > 65535 || k < 0) return ORC_EINVAL;
    int64_t ng = (k + G - 1) / G;
    for (int32_t c = 0; c < C; ++c)
        for (int64_t j = 0; j < k; ++j) {
            int64_t g = j / G;
            int b = bw[(int64_t)c * ng + g];
            float mn = gmin[(int64_t)c * ng + g], mx = gmax[(int64_t)c * ng + g];
            float S, Z;
            orc_group_params(mn, mx, b, &S, &Z);
            out[(int64_t)c * k + j] = orc_value(codes[(int64_t)c * k + j], mn, S, Z);
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Nearest-codeword assignment for the vector-quantized higher-degree SH     */
/* (section "Clustering 1+D SH Coefficients"): idx_i = argmin_j ||x_i-c_j||^2 */
/* with the squared distance summed in FP64 over the dimensions in order;   */
/* ties go to the smallest codeword index.                                   */
/* ------------------------------------------------------------------------ */
int orc_vq_assign(const float* x, int64_t n, int32_t D, const float* cb, int32_t K,
                  int32_t* idx, double* dist) {
    if (n < 0 || D < 1 || K < 1) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float* xi = x + i * D;
        double best = INFINITY;
        int32_t arg = 0;
        for (int32_t j = 0; j < K; ++j) {
            const float* cj = cb + (int64_t)j * D;
            double s = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double diff = (double)xi[d] - (double)cj[d];
                s += diff * diff;
            }
            if (s < best) { best = s; arg = j; }
        }
        idx[i] = arg;
        if (dist) dist[i] = best;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The 0-1 ILP of the bit allocation (equation "ilp"): minimize the summed   */
/* loss of the chosen options, one option per class (block), subject to the */
/* summed size <= budget.  Among optimal solutions: smaller total size, then */
/* the lexicographically smallest option vector (class 0 first).            */
/* ------------------------------------------------------------------------ */

/* Exhaustive enumeration; only for tiny instances (nopt^ncls small). */
int orc_ilp_exhaustive(const double* err, const int64_t* size, int64_t ncls, int32_t nopt,
                       int64_t budget, uint8_t* choice, double* obj, int64_t* used) {
    if (ncls < 1 || ncls > 8 || nopt < 1 || nopt > 16) return ORC_EINVAL;
    int32_t cur[8] = {0};
    int found = 0;
    double best_obj = 0.0;
    int64_t best_size = 0;
    for (;;) {
        double o = 0.0;
        int64_t s = 0;
        for (int64_t c = 0; c < ncls; ++c) {
            o += err[c * nopt + cur[c]];
            s += size[c * nopt + cur[c]];
        }
        if (s <= budget && (!found || o < best_obj || (o == best_obj && s < best_size))) {
            found = 1;
            best_obj = o;
            best_size = s;
            for (int64_t c = 0; c < ncls; ++c) choice[c] = (uint8_t)cur[c];
        }
        /* next vector in lexicographic order, last class fastest */
        int64_t c = ncls - 1;
        while (c >= 0 && cur[c] == nopt - 1) { cur[c] = 0; --c; }
        if (c < 0) break;
        cur[c] += 1;
    }
    if (!found) return ORC_EINFEASIBLE;
    *obj = best_obj;
    *used = best_size;
    return ORC_OK;
}

/*
 * Dynamic programming over the integer capacity, backwards over the
 * classes: f[c][w] = best (loss, size) of classes c..ncls-1 with total size
 * at most w.  Exact for any instance whose budget fits in memory.
 */
int orc_ilp_dp(const double* err, const int64_t* size, int64_t ncls, int32_t nopt,
               int64_t budget, uint8_t* choice, double* obj, int64_t* used) {
    if (ncls < 1 || nopt < 1 || nopt > 255 || budget < 0) return ORC_EINVAL;
    if (budget > 50000000 || (double)ncls * (double)(budget + 1) > 4e9) return ORC_EINVAL;
    for (int64_t i = 0; i < ncls * nopt; ++i)
        if (size[i] < 0) return ORC_EINVAL;
    int64_t W = budget + 1;
    double* fo = (double*)malloc(sizeof(double) * (size_t)W);
    int64_t* fs = (int64_t*)malloc(sizeof(int64_t) * (size_t)W);
    double* go = (double*)malloc(sizeof(double) * (size_t)W);
    int64_t* gs = (int64_t*)malloc(sizeof(int64_t) * (size_t)W);
    uint8_t* pick = (uint8_t*)malloc((size_t)ncls * (size_t)W);
    if (!fo || !fs || !go || !gs || !pick) {
        free(fo); free(fs); free(go); free(gs); free(pick);
        return ORC_ENOMEM;
    }
    /* empty suffix: loss 0, size 0, feasible for every capacity */
    for (int64_t w = 0; w < W; ++w) { fo[w] = 0.0; fs[w] = 0; }
    for (int64_t c = ncls - 1; c >= 0; --c) {
        for (int64_t w = 0; w < W; ++w) {
            double bo = INFINITY;
            int64_t bs = 0;
            int32_t bj = -1;
            for (int32_t j = 0; j < nopt; ++j) {
                int64_t s = size[c * nopt + j];
                if (s > w) continue;
                double ro = fo[w - s];
                if (isinf(ro)) continue;
                double o = err[c * nopt + j] + ro;
                int64_t ts = s + fs[w - s];
                if (bj < 0 || o < bo || (o == bo && ts < bs)) { bo = o; bs = ts; bj = j; }
            }
            go[w] = bj < 0 ? INFINITY : bo;
            gs[w] = bs;
            pick[c * W + w] = bj < 0 ? 255 : (uint8_t)bj;
        }
        double* to = fo; fo = go; go = to;
        int64_t* ts = fs; fs = gs; gs = ts;
    }
    int status = ORC_OK;
    if (isinf(fo[budget])) {
        status = ORC_EINFEASIBLE;
    } else {
        int64_t w = budget;
        int64_t total = 0;
        double o = 0.0;
        for (int64_t c = 0; c < ncls; ++c) {
            uint8_t j = pick[c * W + w];
            choice[c] = j;
            w -= size[c * nopt + j];
            total += size[c * nopt + j];
            o += err[c * nopt + j];
        }
        *obj = o;
        *used = total;
    }
    free(fo); free(fs); free(go); free(gs); free(pick);
    return status;
}
