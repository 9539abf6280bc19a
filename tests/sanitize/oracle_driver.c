/* Drives every entry point of the C oracle on random and edge-case inputs,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure).  Exits non-zero when a call returns an unexpected status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_prune_select(const float* imp, int64_t n, const int64_t* k, int32_t T, int32_t* kept);
int64_t orc_hist_bins(const uint8_t* bl, int32_t nb);
int orc_quant_sweep(const float* attr, int64_t ld, int32_t C, int64_t N, const float* imp,
                    const int32_t* kept, const int64_t* k, int32_t T, int32_t G, const uint8_t* bl,
                    int32_t nb, double* err, double* bits, float* gmin, float* gmax, uint32_t* hist);
int orc_quantize(const float* attr, int64_t ld, int32_t C, int64_t N, const int32_t* kept, int64_t k,
                 int32_t G, const uint8_t* bw, uint16_t* codes, float* gmin, float* gmax);
int orc_dequantize(const uint16_t* codes, int64_t k, int32_t C, int32_t G, const uint8_t* bw,
                   const float* gmin, const float* gmax, float* out);
int orc_vq_assign(const float* x, int64_t n, int32_t D, const float* cb, int32_t K, int32_t* idx,
                  double* dist);
int orc_ilp_exhaustive(const double* err, const int64_t* size, int64_t ncls, int32_t nopt, int64_t budget,
                       uint8_t* choice, double* obj, int64_t* used);
int orc_ilp_dp(const double* err, const int64_t* size, int64_t ncls, int32_t nopt, int64_t budget,
               uint8_t* choice, double* obj, int64_t* used);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) {
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
static void expect(int got, int want, const char* what) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d\n", what, got, want);
        ++fails;
    }
}

static void sweep_case(int64_t N, int32_t C, int32_t G, const uint8_t* bl, int32_t nb, int nan_at) {
    float* attr = malloc(sizeof(float) * (size_t)(N * C + 1));
    float* imp = malloc(sizeof(float) * (size_t)(N + 1));
    for (int64_t i = 0; i < N * C; ++i) attr[i] = (float)(urand() * 4.0 - 2.0);
    for (int64_t i = 0; i < N; ++i) imp[i] = (float)(urand() < 0.1 ? 0.0 : exp(urand() * 4.0 - 2.0));
    if (C > 1)
        for (int64_t i = 0; i < N; ++i) attr[N + i] = 1.5f; /* a constant channel */
    if (nan_at >= 0 && nan_at < N * C) attr[nan_at] = NAN;
    int64_t k[4] = {0, N, N / 3, N > 0 ? 1 : 0};
    int32_t T = 4;
    int64_t ksum = 0, kmax = 0;
    for (int t = 0; t < T; ++t) {
        ksum += k[t];
        if (k[t] > kmax) kmax = k[t];
    }
    int32_t* kept = malloc(sizeof(int32_t) * (size_t)(ksum + 1));
    expect(orc_prune_select(imp, N, k, T, kept), 0, "prune_select");
    int64_t gm = (kmax + G - 1) / G;
    int64_t hb = orc_hist_bins(bl, nb);
    size_t slots = (size_t)(T * C * (gm > 0 ? gm : 1));
    double* err = malloc(sizeof(double) * slots * nb);
    double* bits = malloc(sizeof(double) * slots * nb);
    float* mn = malloc(sizeof(float) * slots);
    float* mx = malloc(sizeof(float) * slots);
    uint32_t* hist = malloc(sizeof(uint32_t) * slots * (size_t)hb);
    int rc = orc_quant_sweep(attr, N, C, N, imp, kept, k, T, G, bl, nb, err, bits, mn, mx, hist);
    expect(rc, nan_at >= 0 ? -2 : 0, "quant_sweep");
    if (nan_at < 0) {
        int64_t kk = k[2];
        int64_t ng = (kk + G - 1) / G;
        uint8_t* bw = malloc((size_t)(C * ng + 1));
        for (int64_t i = 0; i < C * ng; ++i) bw[i] = bl[(int)(urand() * nb) % nb];
        uint16_t* codes = malloc(sizeof(uint16_t) * (size_t)(C * kk + 1));
        float* qmn = malloc(sizeof(float) * (size_t)(C * ng + 1));
        float* qmx = malloc(sizeof(float) * (size_t)(C * ng + 1));
        float* out = malloc(sizeof(float) * (size_t)(C * kk + 1));
        const int32_t* kt = kept + k[0] + k[1];
        expect(orc_quantize(attr, N, C, N, kt, kk, G, bw, codes, qmn, qmx), 0, "quantize");
        expect(orc_dequantize(codes, kk, C, G, bw, qmn, qmx, out), 0, "dequantize");
        free(bw);
        free(codes);
        free(qmn);
        free(qmx);
        free(out);
    }
    free(attr);
    free(imp);
    free(kept);
    free(err);
    free(bits);
    free(mn);
    free(mx);
    free(hist);
}

int main(void) {
    const uint8_t all[16] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
    const uint8_t few[3] = {2, 9, 16};
    sweep_case(3000, 3, 256, all, 16, -1);
    sweep_case(5000, 2, 4097, few, 3, -1);
    sweep_case(777, 4, 1, few, 3, -1);
    sweep_case(1, 1, 7, all, 16, -1);
    sweep_case(2000, 3, 100, few, 3, 2000 * 2 + 17);
    /* invalid arguments are refused before any access */
    expect(orc_quant_sweep(NULL, 0, 0, 0, NULL, NULL, NULL, 0, 0, few, 3, NULL, NULL, NULL, NULL, NULL), -1,
           "quant_sweep(C=0)");
    /* nearest codeword */
    {
        const int n = 500, D = 7, K = 33;
        float* x = malloc(sizeof(float) * n * D);
        float* cb = malloc(sizeof(float) * K * D);
        for (int i = 0; i < n * D; ++i) x[i] = (float)(urand() - 0.5);
        for (int i = 0; i < K * D; ++i) cb[i] = (float)(urand() - 0.5);
        int32_t* idx = malloc(sizeof(int32_t) * n);
        double* dist = malloc(sizeof(double) * n);
        expect(orc_vq_assign(x, n, D, cb, K, idx, dist), 0, "vq_assign");
        expect(orc_vq_assign(x, 0, D, cb, K, idx, dist), 0, "vq_assign(n=0)");
        free(x);
        free(cb);
        free(idx);
        free(dist);
    }
    /* exact 0-1 ILPs: enumeration and DP, feasible and infeasible budgets */
    {
        const int ncls = 6, nopt = 5;
        double err[30];
        int64_t size[30];
        for (int i = 0; i < ncls * nopt; ++i) {
            err[i] = urand() * 10.0;
            size[i] = 1 + (int64_t)(urand() * 50.0);
        }
        uint8_t ch[8];
        double obj;
        int64_t used;
        expect(orc_ilp_exhaustive(err, size, ncls, nopt, 150, ch, &obj, &used), 0, "ilp_exhaustive");
        expect(orc_ilp_dp(err, size, ncls, nopt, 150, ch, &obj, &used), 0, "ilp_dp");
        expect(orc_ilp_dp(err, size, ncls, nopt, 0, ch, &obj, &used), -3, "ilp_dp(infeasible)");
        expect(orc_ilp_exhaustive(err, size, 9, nopt, 150, ch, &obj, &used), -1, "ilp_exhaustive(9 classes)");
    }
    if (fails) return 1;
    printf("oracle driver: ok\n");
    return 0;
}
