// Drives the host side of the library (exact 0-1 ILP, size tables, the
// reserve-ratio search, the hierarchical solver and the calibrated search)
// on random and edge-case tables, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure).  Exits non-zero when a
// call returns an unexpected status or breaks its budget.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "mgs.h"

static int fails = 0;
static void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "failed: %s\n", what);
        ++fails;
    }
}

int main() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    // plain instances of several sizes: optimum within the budget, exact ties
    for (int rep = 0; rep < 6; ++rep) {
        const int64_t ncls = 20 + rep * 300;
        const int nopt = 1 + rep * 3;
        std::vector<double> err(ncls * nopt);
        std::vector<int64_t> size(ncls * nopt);
        int64_t smin = 0, smax = 0;
        for (int64_t c = 0; c < ncls; ++c) {
            double e = 100.0 * u(rng) + 1.0;
            int64_t s = 10 + (int64_t)(u(rng) * 5);
            int64_t lo = INT64_MAX, hi = 0;
            for (int o = 0; o < nopt; ++o) {
                err[c * nopt + o] = rep == 2 ? 1.0 : e;  // rep 2: every option ties
                size[c * nopt + o] = s;
                lo = std::min(lo, s);
                hi = std::max(hi, s);
                e *= 0.5 + 0.4 * u(rng);
                s += 1 + (int64_t)(u(rng) * 30);
            }
            smin += lo;
            smax += hi;
        }
        std::vector<uint8_t> choice(ncls);
        double obj = 0.0;
        int64_t used = 0;
        const int64_t budget = smin + (smax - smin) / 3;
        int rc = mgs_ilp_solve(err.data(), size.data(), ncls, nopt, budget, choice.data(), &obj, &used);
        expect(rc == MGS_OK && used <= budget, "ilp_solve");
        rc = mgs_ilp_solve(err.data(), size.data(), ncls, nopt, smin - 1, choice.data(), &obj, &used);
        expect(rc == MGS_EINFEASIBLE, "ilp_solve(infeasible)");
    }
    // invalid tables
    {
        double err[4] = {1.0, NAN, 2.0, 3.0};
        int64_t size[4] = {1, 2, 3, 4};
        uint8_t ch[2];
        double obj;
        int64_t used;
        expect(mgs_ilp_solve(err, size, 2, 2, 10, ch, &obj, &used) == MGS_EINVAL, "ilp_solve(nan)");
        expect(mgs_ilp_solve(err, size, 2, 0, 10, ch, &obj, &used) == MGS_EINVAL, "ilp_solve(nopt=0)");
    }
    // the reserve-ratio search over sweep-shaped tables, both size rules, the
    // hierarchical solver and the calibrated search
    {
        const int C = 5, G = 64, T = 4;
        const uint8_t bl[4] = {2, 4, 8, 12};
        const int nb = 4;
        const int64_t N = 3000;
        int64_t k[T] = {600, 1200, 2100, 3000};
        const int64_t gm = (3000 + G - 1) / G;
        std::vector<double> err(T * C * gm * nb, NAN), bits(T * C * gm * nb, NAN);
        for (int t = 0; t < T; ++t)
            for (int c = 0; c < C; ++c)
                for (int64_t g = 0; g < (k[t] + G - 1) / G; ++g) {
                    const int64_t n = std::min<int64_t>(G, k[t] - g * G);
                    double e = 50.0 * u(rng) + 1.0;
                    for (int b = 0; b < nb; ++b) {
                        const int64_t i = ((t * C + c) * gm + g) * nb + b;
                        err[i] = e;
                        e *= 0.3 * u(rng) + 0.1;
                        bits[i] = n * bl[b] * (0.5 + 0.4 * u(rng));
                    }
                }
        mgs_sweep_desc d{N, N, C, T, G, nb, k, bl};
        const int64_t budget = N * C * 32 / 12;
        std::vector<uint8_t> best(C * gm);
        std::vector<double> obj(T);
        std::vector<int64_t> used(T), actual(T);
        std::vector<int32_t> st(T), iters(T);
        int32_t bt = -1;
        for (int mode = 0; mode < 2; ++mode)
            for (int flags = 0; flags < 2; ++flags) {
                int rc = mgs_search(&d, err.data(), bits.data(), budget, mode, 4, flags, &bt, best.data(), obj.data(),
                                    used.data(), st.data());
                expect(rc == MGS_OK && bt >= 0 && used[bt] <= budget, "search");
            }
        const int64_t ng = (k[bt] + G - 1) / G;
        std::vector<double> e(C * ng * nb);
        std::vector<int64_t> sz(C * ng * nb);
        std::vector<double> bb(C * ng * nb);
        std::vector<int64_t> nper(C * ng);
        for (int c = 0; c < C; ++c)
            for (int64_t g = 0; g < ng; ++g) {
                nper[c * ng + g] = std::min<int64_t>(G, k[bt] - g * G);
                for (int b = 0; b < nb; ++b) {
                    const int64_t i = ((bt * C + c) * gm + g) * nb + b;
                    e[(c * ng + g) * nb + b] = err[i];
                    bb[(c * ng + g) * nb + b] = bits[i];
                }
            }
        expect(mgs_size_table(bb.data(), nper.data(), C * ng, nb, bl, 0, sz.data()) == MGS_OK, "size_table");
        std::vector<uint8_t> ch(C * ng), cbits(C);
        std::vector<int64_t> cbud(C);
        double o = 0.0;
        int64_t us = 0;
        int rc = mgs_ilp_hierarchical(e.data(), sz.data(), C, ng, nb, bl, budget, ch.data(), &o, &us, cbits.data(),
                                      cbud.data());
        expect((rc == MGS_OK && us <= budget) || rc == MGS_EINFEASIBLE, "ilp_hierarchical");
        rc = mgs_search_calibrated(&d, err.data(), bits.data(), budget, 50000, 16, 4, &bt, best.data(), obj.data(),
                                   actual.data(), iters.data(), st.data());
        expect(rc == MGS_OK || rc == MGS_EINFEASIBLE, "search_calibrated");
    }
    if (fails) return 1;
    std::printf("host ILP driver: ok\n");
    return 0;
}
