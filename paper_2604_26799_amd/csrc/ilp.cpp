// Host side of the search: the exact 0-1 ILP of the bit allocation and the
// reserve-ratio loop around it.
//
// Paper: equation "ilp" (section "Solve the MINLP") -- one bit-width option
// per block (one-hot), minimise the summed quality loss subject to the
// estimated size <= budget; the search algorithm iterates over a discrete
// set of reserve ratios, skips a ratio whose doubled 8-bit size is below the
// budget, and keeps the best configuration.
//
// The ILP is a multiple-choice knapsack.  Exact method:
//   1. drop dominated options (no smaller loss for no larger size);
//   2. LP relaxation on the lower convex hull of each class: greedy over the
//      hull increments by efficiency gives the Lagrange multiplier lambda of
//      the size constraint, a lower bound L(lambda) and an integer
//      incumbent (improved by single-class moves);
//   3. reduced costs r = (err + lambda size) - min over the class: any
//      solution costs at least L(lambda) + sum of its reduced costs, so an
//      option with r > incumbent - L(lambda) is in no solution at least as
//      good as the incumbent;
//   4. expanding core: dynamic programming over (size, loss) states with
//      dominance pruning and the Lagrangian bound, first over the classes
//      whose alternatives are cheapest (beam-limited, to improve the
//      incumbent and so shrink the gap), then exactly over every class that
//      can still change; the others keep their Lagrangian-best option.
// Among optimal solutions the smaller total size wins, then the smaller
// option index in class order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include <omp.h>

#include "../../include/mgs.h"

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
constexpr size_t kStateCap = 20u * 1000u * 1000u;
constexpr size_t kBeam = 20000;  // states per layer in the incumbent passes

struct Opt {
    double e;
    int64_t s;
    int j;
};

struct State {
    int64_t w;     // size used by the core classes so far
    double z;      // loss of the core classes so far
    int32_t prev;  // index of the parent state in the previous layer
    int16_t opt;   // option index (original) chosen for this layer's class
};

// Lexicographic comparison of two DP paths (class order, option index).
bool path_less(const std::vector<std::vector<State>>& layers, size_t layer, int32_t a, int32_t b) {
    // walk both paths back to the first layer, remember the choices
    std::vector<int16_t> pa, pb;
    for (size_t l = layer + 1; l-- > 0;) {
        pa.push_back(layers[l][a].opt);
        pb.push_back(layers[l][b].opt);
        a = layers[l][a].prev;
        b = layers[l][b].prev;
    }
    for (size_t i = pa.size(); i-- > 0;)
        if (pa[i] != pb[i]) return pa[i] < pb[i];
    return false;
}

// Dynamic programming over the classes of a core (in the given order) on
// (size, loss) states: dominated states are dropped, states whose Lagrangian
// bound exceeds UB are pruned, and with beam > 0 only the `beam` states of
// best bound survive a layer (a heuristic pass).  Writes the option index of
// every core class of the best final state (least loss, then least size,
// then lexicographically smallest path).
int core_dp(const std::vector<std::vector<Opt>>& opts, double e_fixed, int64_t cap, double lambda,
            double UB, double tol, size_t beam, std::vector<int16_t>& pick) {
    const size_t n = opts.size();
    if (cap < 0) return MGS_EINFEASIBLE;
    std::vector<double> mr(n + 1, 0.0);  // suffix sums of min(e + lambda s)
    for (size_t i = n; i-- > 0;) {
        double m = kInf;
        for (const Opt& x : opts[i]) m = std::min(m, x.e + lambda * (double)x.s);
        mr[i] = mr[i + 1] + m;
    }
    std::vector<std::vector<State>> layers;
    std::vector<State> cur{{0, 0.0, -1, -1}};
    std::vector<State> nxt;
    size_t total_states = 1;
    for (size_t li = 0; li < n; ++li) {
        nxt.clear();
        for (int32_t si = 0; si < (int32_t)cur.size(); ++si) {
            const State& st = cur[si];
            for (const Opt& x : opts[li]) {
                int64_t w = st.w + x.s;
                if (w > cap) continue;
                double z = st.z + x.e;
                double lb = e_fixed + z + mr[li + 1] - lambda * (double)(cap - w);
                if (lb > UB + tol) continue;
                nxt.push_back({w, z, si, (int16_t)x.j});
            }
        }
        layers.push_back(cur);
        std::sort(nxt.begin(), nxt.end(), [](const State& a, const State& b) {
            if (a.w != b.w) return a.w < b.w;
            return a.z < b.z;
        });
        cur.clear();
        for (size_t i = 0; i < nxt.size(); ++i) {
            const State& st = nxt[i];
            if (!cur.empty()) {
                State& last = cur.back();
                if (st.z > last.z) continue;
                if (st.z == last.z) {
                    // same loss with more size is dominated; same (size, loss) keeps
                    // the lexicographically smaller path: parents first, then option
                    if (st.w == last.w) {
                        bool less = st.prev == last.prev
                                        ? st.opt < last.opt
                                        : path_less(layers, layers.size() - 1, st.prev, last.prev);
                        if (less) last = st;
                    }
                    continue;
                }
            }
            cur.push_back(st);
        }
        if (beam && cur.size() > beam) {
            std::nth_element(cur.begin(), cur.begin() + beam, cur.end(), [&](const State& a, const State& b) {
                return a.z + lambda * (double)a.w < b.z + lambda * (double)b.w;
            });
            cur.resize(beam);
        }
        total_states += cur.size();
        if (total_states > kStateCap) return MGS_ELIMIT;
        if (cur.empty()) return MGS_EINFEASIBLE;
    }
    // least loss; among equal loss the dominance pass kept the least size
    int32_t best = 0;
    for (int32_t i = 1; i < (int32_t)cur.size(); ++i)
        if (cur[i].z < cur[best].z || (cur[i].z == cur[best].z && cur[i].w < cur[best].w)) best = i;
    pick.assign(n, 0);
    layers.push_back(cur);
    int32_t si = best;
    for (size_t li = n; li-- > 0;) {
        const State& st = layers[li + 1][si];
        pick[li] = st.opt;
        si = st.prev;
    }
    return MGS_OK;
}

int solve(const double* err, const int64_t* size, int64_t ncls, int nopt, int64_t budget,
          uint8_t* choice, double* obj, int64_t* used) {
    // ---- 1. per-class options without dominated ones, sorted by size
    std::vector<std::vector<Opt>> cls(ncls);
    int64_t min_total = 0;
    for (int64_t c = 0; c < ncls; ++c) {
        std::vector<Opt> o;
        o.reserve(nopt);
        for (int j = 0; j < nopt; ++j) o.push_back({err[c * nopt + j], size[c * nopt + j], j});
        std::sort(o.begin(), o.end(), [](const Opt& a, const Opt& b) {
            if (a.s != b.s) return a.s < b.s;
            if (a.e != b.e) return a.e < b.e;
            return a.j < b.j;
        });
        std::vector<Opt> keep;
        for (const Opt& x : o)
            if (keep.empty() || x.e < keep.back().e) keep.push_back(x);
        min_total += keep.front().s;
        cls[c] = std::move(keep);
    }
    if (min_total > budget) return MGS_EINFEASIBLE;
    // unconstrained optimum (last option of each class) fits: done
    {
        int64_t tot = 0;
        for (auto& k : cls) tot += k.back().s;
        if (tot <= budget) {
            double o = 0;
            for (int64_t c = 0; c < ncls; ++c) {
                choice[c] = (uint8_t)cls[c].back().j;
                o += cls[c].back().e;
            }
            *obj = o;
            *used = tot;
            return MGS_OK;
        }
    }

    // ---- 2. LP relaxation via hull increments
    struct Inc {
        double eff;  // loss decrease per unit of size
        int64_t c;
        int from, to;  // positions in cls[c]
    };
    std::vector<Inc> incs;
    for (int64_t c = 0; c < ncls; ++c) {
        const auto& o = cls[c];
        std::vector<int> hull{0};
        for (int i = 1; i < (int)o.size(); ++i) {
            while (hull.size() >= 2) {
                const Opt& a = o[hull[hull.size() - 2]];
                const Opt& b = o[hull.back()];
                // drop b if it lies on or above the segment a -> o[i]
                double lhs = (b.e - a.e) * (double)(o[i].s - a.s);
                double rhs = (o[i].e - a.e) * (double)(b.s - a.s);
                if (lhs >= rhs) hull.pop_back();
                else break;
            }
            hull.push_back(i);
        }
        for (size_t h = 1; h < hull.size(); ++h) {
            const Opt& a = o[hull[h - 1]];
            const Opt& b = o[hull[h]];
            incs.push_back({(a.e - b.e) / (double)(b.s - a.s), c, hull[h - 1], hull[h]});
        }
    }
    std::stable_sort(incs.begin(), incs.end(), [](const Inc& a, const Inc& b) { return a.eff > b.eff; });
    std::vector<int> pos(ncls, 0);  // current option position per class
    int64_t cap = budget - min_total;
    double lambda = 0.0;
    bool split = false;
    for (const Inc& in : incs) {
        if (pos[in.c] != in.from) continue;  // (cannot happen for a convex hull)
        int64_t ds = cls[in.c][in.to].s - cls[in.c][in.from].s;
        if (ds <= cap) {
            cap -= ds;
            pos[in.c] = in.to;
        } else {
            lambda = in.eff;
            split = true;
            break;
        }
    }
    if (!split) lambda = 0.0;
    // incumbent: greedy solution improved by single-class moves
    std::vector<int> inc_pos = pos;
    {
        bool improved = true;
        int rounds = 0;
        while (improved && rounds++ < 8) {
            improved = false;
            for (int64_t c = 0; c < ncls; ++c) {
                const auto& o = cls[c];
                int best = inc_pos[c];
                double gain = 0.0;
                for (int i = 0; i < (int)o.size(); ++i) {
                    int64_t ds = o[i].s - o[inc_pos[c]].s;
                    double de = o[inc_pos[c]].e - o[i].e;
                    if (ds <= cap && de > gain) {
                        gain = de;
                        best = i;
                    }
                }
                if (best != inc_pos[c]) {
                    cap -= o[best].s - o[inc_pos[c]].s;
                    inc_pos[c] = best;
                    improved = true;
                }
            }
        }
    }
    double UB = 0.0;
    for (int64_t c = 0; c < ncls; ++c) UB += cls[c][inc_pos[c]].e;

    // ---- 3. Lagrangian bound, reduced costs, Lagrangian-best option per class
    std::vector<double> mlam(ncls);
    std::vector<int> lagbest(ncls, 0);
    double LB0 = -lambda * (double)budget;
    double scale = std::fabs(UB);
    for (int64_t c = 0; c < ncls; ++c) {
        double m = kInf;
        for (int i = 0; i < (int)cls[c].size(); ++i) {
            double v = cls[c][i].e + lambda * (double)cls[c][i].s;
            if (v < m) {  // options are sorted by size: ties keep the smaller size
                m = v;
                lagbest[c] = i;
            }
        }
        mlam[c] = m;
        LB0 += m;
        scale = std::max(scale, std::fabs(m));
    }
    const double tol = 1e-9 * (scale + std::fabs(LB0) + std::fabs(lambda * (double)budget)) + 1e-300;
    // smallest reduced cost of any other option of the class
    std::vector<double> rcmin(ncls, kInf);
    for (int64_t c = 0; c < ncls; ++c)
        for (int i = 0; i < (int)cls[c].size(); ++i)
            if (i != lagbest[c])
                rcmin[c] = std::min(rcmin[c], cls[c][i].e + lambda * (double)cls[c][i].s - mlam[c]);
    std::vector<int64_t> order(ncls);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return rcmin[a] < rcmin[b]; });

    // ---- 4. expanding core: DP over the classes whose alternatives are
    // cheapest in reduced cost improves the incumbent, which shrinks the gap;
    // once every class that can still change (rcmin <= gap) fits in the core,
    // one exact DP over exactly those classes finishes.
    size_t K = 32;
    for (;;) {
        const double gap = UB - LB0 + tol;
        std::vector<int64_t> need;
        for (int64_t c : order) {
            if (rcmin[c] > gap) break;
            need.push_back(c);
        }
        const bool final_pass = need.size() <= K;
        std::vector<int64_t> core = final_pass ? need : std::vector<int64_t>(order.begin(), order.begin() + K);
        if (final_pass) std::sort(core.begin(), core.end());  // index order for the tie rule
        std::vector<char> in_core(ncls, 0);
        for (int64_t c : core) in_core[c] = 1;
        double e_fixed = 0.0;
        int64_t s_fixed = 0;
        for (int64_t c = 0; c < ncls; ++c)
            if (!in_core[c]) {
                e_fixed += cls[c][lagbest[c]].e;
                s_fixed += cls[c][lagbest[c]].s;
            }
        std::vector<std::vector<Opt>> opts(core.size());
        for (size_t i = 0; i < core.size(); ++i)
            for (const Opt& x : cls[core[i]])
                if (x.e + lambda * (double)x.s - mlam[core[i]] <= gap) opts[i].push_back(x);
        std::vector<int16_t> pick;
        double zb = 0.0;
        int rc = core_dp(opts, e_fixed, budget - s_fixed, lambda, UB, tol,
                         final_pass ? 0 : kBeam, pick);
        if (rc == MGS_ELIMIT) return rc;
        if (final_pass) {
            if (rc != MGS_OK) return MGS_EINFEASIBLE;  // (cannot happen: the incumbent is a state)
            for (int64_t c = 0; c < ncls; ++c)
                if (!in_core[c]) choice[c] = (uint8_t)cls[c][lagbest[c]].j;
            for (size_t i = 0; i < core.size(); ++i) choice[core[i]] = (uint8_t)pick[i];
            break;
        }
        if (rc == MGS_OK) {
            zb = e_fixed;
            for (size_t i = 0; i < core.size(); ++i) zb += err[core[i] * nopt + pick[i]];
            if (zb < UB) UB = zb;
        }
        K *= 4;
    }
    double o = 0.0;
    int64_t u = 0;
    for (int64_t c = 0; c < ncls; ++c) {
        o += err[c * nopt + choice[c]];
        u += size[c * nopt + choice[c]];
    }
    *obj = o;
    *used = u;
    return MGS_OK;
}

}  // namespace

extern "C" int mgs_ilp_solve(const double* h_err, const int64_t* h_size, int64_t ncls, int32_t nopt,
                             int64_t budget, uint8_t* h_choice, double* h_obj, int64_t* h_used) {
    if (ncls < 1 || nopt < 1 || nopt > 255 || !h_err || !h_size || !h_choice || !h_obj || !h_used)
        return MGS_EINVAL;
    for (int64_t i = 0; i < ncls * nopt; ++i)
        if (!std::isfinite(h_err[i]) || h_size[i] < 0) return MGS_EINVAL;
    return solve(h_err, h_size, ncls, nopt, budget, h_choice, h_obj, h_used);
}

static const int kMetaBits = 72;  // two FP32 bounds + one byte of bit-width per group

extern "C" int mgs_size_table(const double* h_bits, const int64_t* h_n, int64_t ncls, int32_t nb,
                              const uint8_t* h_bitlist, int32_t mode, int64_t* h_size) {
    if (ncls < 0 || nb < 1 || !h_size || (mode != 0 && mode != 1)) return MGS_EINVAL;
    if (mode == 0 && !h_bits) return MGS_EINVAL;
    if (mode == 1 && (!h_n || !h_bitlist)) return MGS_EINVAL;
    for (int64_t c = 0; c < ncls; ++c)
        for (int i = 0; i < nb; ++i) {
            if (mode == 0) {
                double b = h_bits[c * nb + i];
                if (!std::isfinite(b) || b < 0) return MGS_EINVAL;
                h_size[c * nb + i] = (int64_t)std::ceil(b) + kMetaBits;
            } else {
                h_size[c * nb + i] = h_n[c] * (int64_t)h_bitlist[i] + kMetaBits;
            }
        }
    return MGS_OK;
}

extern "C" int mgs_search(const mgs_sweep_desc* d, const double* h_err, const double* h_bits,
                          int64_t budget_bits, int32_t size_mode, int32_t threads,
                          int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_used) {
    if (!d || !d->h_k || !d->h_bits || !h_err || !h_bits || !h_best_t || !h_best_bits || !h_obj ||
        !h_used)
        return MGS_EINVAL;
    if (d->C < 1 || d->T < 1 || d->T > MGS_MAX_RATIOS || d->G < 1 || d->nb < 1 ||
        d->nb > MGS_MAX_BITS || (size_mode != 0 && size_mode != 1))
        return MGS_EINVAL;
    const int C = d->C, T = d->T, G = d->G, nb = d->nb;
    int64_t kmax = 0;
    for (int t = 0; t < T; ++t) kmax = std::max(kmax, d->h_k[t]);
    const int64_t gmaxn = (kmax + G - 1) / G;
    int b8 = -1;
    for (int i = 0; i < nb; ++i)
        if (d->h_bits[i] == 8) b8 = i;
    std::vector<int> status(T, MGS_OK);
    std::vector<std::vector<uint8_t>> choice(T);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads > 0 ? threads : omp_get_max_threads())
    for (int t = 0; t < T; ++t) {
        h_obj[t] = std::numeric_limits<double>::quiet_NaN();
        h_used[t] = 0;
        const int64_t k = d->h_k[t];
        const int64_t ng = (k + G - 1) / G;
        const int64_t ncls = (int64_t)C * ng;
        if (ncls == 0) {
            status[t] = MGS_EINFEASIBLE;
            continue;
        }
        std::vector<double> e(ncls * nb), bt(ncls * nb);
        std::vector<int64_t> n(ncls), sz(ncls * nb);
        for (int c = 0; c < C; ++c)
            for (int64_t g = 0; g < ng; ++g) {
                int64_t cls = (int64_t)c * ng + g;
                int64_t slot = ((int64_t)t * C + c) * gmaxn + g;
                n[cls] = std::min<int64_t>(G, k - g * G);
                for (int i = 0; i < nb; ++i) {
                    e[cls * nb + i] = h_err[slot * nb + i];
                    bt[cls * nb + i] = h_bits[slot * nb + i];
                }
            }
        int rc = mgs_size_table(bt.data(), n.data(), ncls, nb, d->h_bits, size_mode, sz.data());
        if (rc) {
            status[t] = rc;
            continue;
        }
        // size of the all-8-bit configuration
        int64_t s8 = 0;
        for (int64_t cls = 0; cls < ncls; ++cls)
            s8 += (b8 >= 0) ? sz[cls * nb + b8] : n[cls] * 8 + kMetaBits;
        if (2 * s8 < budget_bits) {
            status[t] = MGS_EINFEASIBLE;
            continue;
        }
        choice[t].resize(ncls);
        double o = 0;
        int64_t u = 0;
        rc = mgs_ilp_solve(e.data(), sz.data(), ncls, nb, budget_bits, choice[t].data(), &o, &u);
        status[t] = rc;
        if (rc == MGS_OK) {
            h_obj[t] = o;
            h_used[t] = u;
        }
    }
    for (int t = 0; t < T; ++t)
        if (status[t] != MGS_OK && status[t] != MGS_EINFEASIBLE) return status[t];
    int best = -1;
    for (int t = 0; t < T; ++t) {
        if (status[t] != MGS_OK) continue;
        if (best < 0 || h_obj[t] < h_obj[best] ||
            (h_obj[t] == h_obj[best] &&
             (d->h_k[t] > d->h_k[best] || (d->h_k[t] == d->h_k[best] && t > best))))
            best = t;
    }
    *h_best_t = best;
    if (best < 0) return MGS_EINFEASIBLE;
    const int64_t ng = (d->h_k[best] + G - 1) / G;
    for (int64_t cls = 0; cls < (int64_t)C * ng; ++cls) h_best_bits[cls] = d->h_bits[choice[best][cls]];
    return MGS_OK;
}
