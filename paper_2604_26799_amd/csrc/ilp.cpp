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
#include <atomic>
#include <cmath>
#include <climits>
#include <cstdint>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include <omp.h>

#include "../../include/mgs.h"

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
constexpr size_t kStateCap = 20u * 1000u * 1000u;
// Incumbent passes (beam width, first core size, largest exact core), tried
// in order: a cheap schedule first; a wider one when the exact pass of the
// cheaper one exceeds the state limit, or would span more classes than the
// schedule's exact core (its weaker incumbent left too large a gap: a wider
// beam over a small core usually closes most of it for a fraction of what
// such an exact pass costs).
constexpr size_t kNoLimit = std::numeric_limits<size_t>::max();
constexpr size_t kWideAfter = 512;  // core size from which a fruitless beam pass hands over
constexpr struct { size_t beam, k0, exact_max; } kSchedules[] = {
    {1000, 32, 400}, {4000, 128, 1600}, {16000, 128, kNoLimit}};

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

// Lower bound on the cost of completing a partial solution from the classes
// not yet processed, as a function of D = the capacity left if those classes
// keep their Lagrangian-best options.  Relative to that default each class
// offers points (dS, r) with r >= 0 the reduced cost; the LP relaxation takes
// segments of each class's lower convex hull in order of cost per bit:
//   D >= 0: h(D) = lambda D - savings of the upgrades cheaper than lambda per
//           bit that fit into D (capacity left unused costs lambda per bit);
//   D <  0: h(D) = cost of the cheapest downgrades freeing -D bits (infinite
//           when they cannot).
// h >= 0, so the Lagrangian bound plus h(D) is still a valid lower bound.
struct Completion {
    struct Seg {
        double slope;  // reduced cost per bit
        int64_t len;   // bits
        int32_t cls;   // core position
    };
    std::vector<Seg> up, down;        // all segments, sorted by slope
    std::vector<int64_t> ulen, dlen;  // cumulative lengths of the live ones
    std::vector<double> usave, dcost, uslope, dslope;
    double lambda = 0.0;

    void build(const std::vector<std::vector<Opt>>& opts, const std::vector<double>& m,
               const std::vector<int64_t>& sdef, double lam) {
        lambda = lam;
        for (size_t i = 0; i < opts.size(); ++i) {
            std::vector<std::pair<int64_t, double>> pu, pd;  // (bits, r) away from the default
            for (const Opt& x : opts[i]) {
                const int64_t ds = x.s - sdef[i];
                const double r = std::max(0.0, x.e + lam * (double)x.s - m[i]);
                if (ds > 0) pu.push_back({ds, r});
                if (ds < 0) pd.push_back({-ds, r});
            }
            add_hull(pu, (int32_t)i, up);
            add_hull(pd, (int32_t)i, down);
        }
        auto by = [](const Seg& a, const Seg& b) { return a.slope < b.slope; };
        std::stable_sort(up.begin(), up.end(), by);
        std::stable_sort(down.begin(), down.end(), by);
    }
    // lower convex hull from (0, 0) of points (bits > 0, r)
    static void add_hull(std::vector<std::pair<int64_t, double>>& pts, int32_t cls, std::vector<Seg>& out) {
        if (pts.empty()) return;
        std::sort(pts.begin(), pts.end());
        std::vector<std::pair<int64_t, double>> h{{0, 0.0}};
        for (const auto& q : pts) {
            while (h.size() >= 2) {
                const auto& a = h[h.size() - 2];
                const auto& b = h.back();
                if ((b.second - a.second) * (double)(q.first - a.first) >=
                    (q.second - a.second) * (double)(b.first - a.first))
                    h.pop_back();
                else
                    break;
            }
            if (q.first == h.back().first) {
                if (q.second < h.back().second) h.back() = q;
                continue;
            }
            h.push_back(q);
        }
        for (size_t k = 1; k < h.size(); ++k) {
            int64_t len = h[k].first - h[k - 1].first;
            out.push_back({(h[k].second - h[k - 1].second) / (double)len, len, cls});
        }
    }
    // keep the segments of classes after position `done`
    void restrict_after(int64_t done) {
        ulen.clear(); usave.clear(); uslope.clear();
        dlen.clear(); dcost.clear(); dslope.clear();
        int64_t L = 0;
        double V = 0.0;
        for (const Seg& g : up) {
            if (g.cls <= done || g.slope >= lambda) continue;
            L += g.len;
            V += (lambda - g.slope) * (double)g.len;
            ulen.push_back(L); usave.push_back(V); uslope.push_back(g.slope);
        }
        L = 0;
        V = 0.0;
        for (const Seg& g : down) {
            if (g.cls <= done) continue;
            L += g.len;
            V += g.slope * (double)g.len;
            dlen.push_back(L); dcost.push_back(V); dslope.push_back(g.slope);
        }
    }
    // Position cursors for evaluating h at monotonically decreasing D (states
    // visited in increasing size): amortised O(1) instead of a binary search.
    struct Cursor {
        size_t ku = SIZE_MAX, kd = 0;
    };
    double h_at(int64_t D, Cursor& c) const {
        if (D >= 0) {
            // first k with ulen[k] >= D; D only decreases, so k only moves down
            if (c.ku == SIZE_MAX) c.ku = ulen.size();
            while (c.ku > 0 && ulen[c.ku - 1] >= D) --c.ku;
            const size_t k = c.ku;
            if (k == ulen.size()) return std::max(0.0, lambda * (double)D - (usave.empty() ? 0.0 : usave.back()));
            double prevL = k ? (double)ulen[k - 1] : 0.0, prevV = k ? usave[k - 1] : 0.0;
            return std::max(0.0, lambda * (double)D - prevV - (lambda - uslope[k]) * ((double)D - prevL));
        }
        // first k with dlen[k] >= F = -D; F only grows, so k only moves up
        const int64_t F = -D;
        while (c.kd < dlen.size() && dlen[c.kd] < F) ++c.kd;
        const size_t k = c.kd;
        if (k == dlen.size()) return kInf;
        double prevL = k ? (double)dlen[k - 1] : 0.0, prevV = k ? dcost[k - 1] : 0.0;
        return prevV + dslope[k] * ((double)F - prevL);
    }
    double h(int64_t D) const {
        if (D >= 0) {
            size_t k = std::lower_bound(ulen.begin(), ulen.end(), D) - ulen.begin();
            if (k == ulen.size()) return std::max(0.0, lambda * (double)D - (usave.empty() ? 0.0 : usave.back()));
            double prevL = k ? (double)ulen[k - 1] : 0.0, prevV = k ? usave[k - 1] : 0.0;
            return std::max(0.0, lambda * (double)D - prevV - (lambda - uslope[k]) * ((double)D - prevL));
        }
        const int64_t F = -D;
        size_t k = std::lower_bound(dlen.begin(), dlen.end(), F) - dlen.begin();
        if (k == dlen.size()) return kInf;
        double prevL = k ? (double)dlen[k - 1] : 0.0, prevV = k ? dcost[k - 1] : 0.0;
        return prevV + dslope[k] * ((double)F - prevL);
    }
};

// Dynamic programming over the classes of a core (in the given order) on
// (size, loss) states kept sorted by size.  A layer is the merge of the
// previous layer shifted by each option's size (every shifted list is
// already sorted), so it costs O(states x options); dominated states are
// dropped during the merge, states whose Lagrangian bound exceeds UB are
// pruned, and with beam > 0 only the `beam` states of best bound survive a
// layer (a heuristic pass).  Writes the option index of every core class of
// the best final state (least loss, then least size, then lexicographically
// smallest path).
int core_dp(const std::vector<std::vector<Opt>>& opts, double e_fixed, int64_t cap, double lambda,
            double UB, double tol, size_t beam, std::vector<int16_t>& pick) {
    const size_t n = opts.size();
    if (cap < 0) return MGS_EINFEASIBLE;
    // per class: Lagrangian minimum m and the size of its (smallest) minimiser
    std::vector<double> m(n, kInf);
    std::vector<int64_t> sdef(n, 0);
    for (size_t i = 0; i < n; ++i)
        for (const Opt& x : opts[i]) {
            const double v = x.e + lambda * (double)x.s;
            if (v < m[i]) {
                m[i] = v;
                sdef[i] = x.s;
            }
        }
    std::vector<double> mr(n + 1, 0.0);  // suffix sums of m
    std::vector<int64_t> sr(n + 1, 0);   // suffix sums of sdef
    for (size_t i = n; i-- > 0;) {
        mr[i] = mr[i + 1] + m[i];
        sr[i] = sr[i + 1] + sdef[i];
    }
    Completion comp;
    comp.build(opts, m, sdef, lambda);
    std::vector<std::vector<State>> layers;
    std::vector<State> cur{{0, 0.0, -1, -1}};
    std::vector<State> nxt;
    std::vector<double> keys;
    size_t total_states = 1;
    for (size_t li = 0; li < n; ++li) {
        const std::vector<Opt>& o = opts[li];
        const int nopt_l = (int)o.size();
        const double rest = e_fixed + mr[li + 1];
        comp.restrict_after((int64_t)li);
        // bound of a state after this layer: Lagrangian part + completion LP
        // (each caller visits states in increasing size through its own cursor)
        auto bound = [&](int64_t w, double z, Completion::Cursor& cu) {
            return rest + z - lambda * (double)(cap - w) + comp.h_at(cap - w - sr[li + 1], cu);
        };
        // k-way merge of cur + o[j] by (size, loss); heap of the list heads
        std::vector<int32_t> head(nopt_l, 0);
        std::vector<Completion::Cursor> cursor(nopt_l);
        auto state_at = [&](int j, int32_t i) {
            return State{cur[i].w + o[j].s, cur[i].z + o[j].e, i, (int16_t)o[j].j};
        };
        auto less = [&](const State& a, const State& b) {
            if (a.w != b.w) return a.w < b.w;
            return a.z < b.z;
        };
        // advance a head past states that overflow the capacity or the bound
        auto valid = [&](int j, int32_t i) {
            const State st = state_at(j, i);
            if (st.w > cap) return 0;  // the list is sorted by size: stop this list
            if (bound(st.w, st.z, cursor[j]) > UB + tol) return 1;  // skip
            return 2;
        };
        auto settle = [&](int j) {
            while (head[j] < (int32_t)cur.size()) {
                int v = valid(j, head[j]);
                if (v == 0) {
                    head[j] = (int32_t)cur.size();
                    break;
                }
                if (v == 2) break;
                ++head[j];
            }
        };
        for (int j = 0; j < nopt_l; ++j) settle(j);
        layers.push_back(cur);
        nxt.clear();
        for (;;) {
            int bj = -1;
            State best{};
            for (int j = 0; j < nopt_l; ++j) {
                if (head[j] >= (int32_t)cur.size()) continue;
                State st = state_at(j, head[j]);
                if (bj < 0 || less(st, best)) {
                    best = st;
                    bj = j;
                }
            }
            if (bj < 0) break;
            ++head[bj];
            settle(bj);
            if (!nxt.empty()) {
                State& last = nxt.back();
                if (best.z > last.z) continue;
                if (best.z == last.z) {
                    // same loss with more size is dominated; same (size, loss) keeps
                    // the lexicographically smaller path: parents first, then option
                    if (best.w == last.w) {
                        bool lt = best.prev == last.prev
                                      ? best.opt < last.opt
                                      : path_less(layers, layers.size() - 1, best.prev, last.prev);
                        if (lt) last = best;
                    }
                    continue;
                }
                if (best.w == last.w) {  // same size, strictly less loss: replace
                    last = best;
                    continue;
                }
            }
            nxt.push_back(best);
        }
        if (beam && nxt.size() > beam) {
            // keep the `beam` states of least bound, in size order
            keys.resize(nxt.size());
            Completion::Cursor cu;
            for (size_t i = 0; i < nxt.size(); ++i) keys[i] = bound(nxt[i].w, nxt[i].z, cu);
            std::vector<double> sel(keys);
            std::nth_element(sel.begin(), sel.begin() + (beam - 1), sel.end());
            const double cut = sel[beam - 1];
            size_t w = 0;
            for (size_t i = 0; i < nxt.size() && w < beam; ++i)
                if (keys[i] <= cut) nxt[w++] = nxt[i];
            nxt.resize(w);
        }
        cur.swap(nxt);
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

// One multiple-choice knapsack instance: prepare() runs the LP relaxation
// (and returns early when the unconstrained optimum fits), exact() the DP.
struct Mckp {
    // writes the nopt options (loss, size, original index) of class c; false
    // if the class's inputs are invalid
    using Fill = std::function<bool(int64_t c, Opt* o)>;
    Fill fill;
    int64_t ncls;
    int nopt;
    int64_t budget;
    // the options of every class without dominated ones, sorted by size,
    // in one array: class c is opt[coff[c] .. coff[c+1])
    std::vector<Opt> opt;
    std::vector<int64_t> coff;
    struct Span {
        const Opt* p;
        int n;
        const Opt& operator[](int i) const { return p[i]; }
        int size() const { return n; }
        const Opt& front() const { return p[0]; }
        const Opt& back() const { return p[n - 1]; }
        const Opt* begin() const { return p; }
        const Opt* end() const { return p + n; }
    };
    Span cls(int64_t c) const { return Span{opt.data() + coff[c], (int)(coff[c + 1] - coff[c])}; }
    // option j (original index) of class c: a chosen option is never a
    // dominated one, so it is among the kept options
    const Opt& opt_j(int64_t c, int j) const {
        const Span o = cls(c);
        for (int i = 0; i + 1 < o.size(); ++i)
            if (o[i].j == j) return o[i];
        return o.back();
    }
    std::vector<int> inc_pos, lagbest;
    std::vector<double> mlam, rcmin;
    std::vector<int64_t> order;
    double lambda = 0.0, LB0 = 0.0, UB = 0.0, tol = 0.0;
    bool trivial = false;  // the unconstrained optimum fits the budget
    std::vector<int> greedy_pos;  // LP greedy solution (its integral part)
    // the LP step's lower hulls and its heap of next increments
    struct Head {
        double eff;
        int64_t c;
        int64_t h;  // index in hv of the increment's end vertex
    };
    struct Inc {
        double eff;
        int64_t ds;  // its size
        int64_t c;
        int64_t h;
    };
    std::vector<int> hv;
    std::vector<int64_t> hoff;
    std::vector<Head> heap;
    std::vector<Inc> inc;  // every hull increment, for the selection
    int64_t greedy_cap = 0;       // capacity it leaves
    bool solve_ready = false;     // phase 2 done

    Mckp(const double* e, const int64_t* s, int64_t n, int o, int64_t b) : ncls(n), nopt(o), budget(b) {
        fill = [e, s, o](int64_t c, Opt* x) {
            for (int j = 0; j < o; ++j) x[j] = {e[c * o + j], s[c * o + j], j};
            return true;
        };
    }
    Mckp(Fill f, int64_t n, int o, int64_t b) : fill(std::move(f)), ncls(n), nopt(o), budget(b) {}
    Mckp() : ncls(0), nopt(0), budget(0) {}

    // Another instance in the same object: the arrays keep their capacity, so
    // a long-lived object bounds one instance after another without fresh
    // allocations.  Only prepare_bound may follow.
    void rebind(Fill f, int64_t n, int o, int64_t b) {
        fill = std::move(f);
        ncls = n;
        nopt = o;
        budget = b;
        lambda = LB0 = UB = tol = 0.0;
        trivial = false;
        solve_ready = false;
        greedy_cap = 0;
    }

    // Lower bound on the optimum (the optimum itself when trivial).
    double lower_bound() const { return LB0; }

    // Both phases (the single-instance solver).
    int prepare() {
        int rc = prepare_bound();
        if (rc == MGS_OK && !trivial) prepare_solve();
        return rc;
    }

    // Phase 1, enough for the lower bound: options without dominated ones,
    // the LP relaxation (lambda) and the Lagrangian bound.
    int prepare_bound() {
    // ---- 1. per-class options without dominated ones, sorted by size
    opt.clear();
    opt.reserve((size_t)ncls * nopt);
    coff.assign(ncls + 1, 0);
    int64_t min_total = 0, max_total = 0;
    double max_obj = 0.0;
    Opt o[256];
    for (int64_t c = 0; c < ncls; ++c) {
        if (!fill(c, o)) return MGS_EINVAL;
        // insertion sort by (size, loss, index): the options of a class are
        // few and nearly sorted already (sizes grow with the bit-width)
        for (int i = 1; i < nopt; ++i) {
            const Opt x = o[i];
            int k = i;
            while (k > 0 && (o[k - 1].s > x.s || (o[k - 1].s == x.s && (o[k - 1].e > x.e ||
                                                                         (o[k - 1].e == x.e && o[k - 1].j > x.j))))) {
                o[k] = o[k - 1];
                --k;
            }
            o[k] = x;
        }
        const size_t first = opt.size();
        for (int i = 0; i < nopt; ++i)
            if (opt.size() == first || o[i].e < opt.back().e) opt.push_back(o[i]);
        coff[c + 1] = (int64_t)opt.size();
        min_total += opt[first].s;
        max_total += opt.back().s;
        max_obj += opt.back().e;
    }
    if (min_total > budget) return MGS_EINFEASIBLE;
    // unconstrained optimum (last option of each class) fits: done
    if (max_total <= budget) {
        trivial = true;
        LB0 = UB = max_obj;
        return MGS_OK;
    }

    // ---- 2. LP relaxation: greedy over the lower-hull increments of all
    // classes by decreasing efficiency (loss saved per bit), ties by class and
    // hull position, until one does not fit; its efficiency is lambda.  Each
    // class's increments are already in decreasing efficiency (convex hull),
    // so a heap merge of the classes yields that order and stops at the split.
    hv.clear();                      // hull vertices (option positions), all classes
    hoff.assign(ncls + 1, 0);        // class c: hv[hoff[c] .. hoff[c+1])
    hv.reserve((size_t)ncls * 4);
    for (int64_t c = 0; c < ncls; ++c) {
        const auto& o = cls(c);
        const size_t h0 = hv.size();
        hv.push_back(0);
        for (int i = 1; i < (int)o.size(); ++i) {
            while (hv.size() - h0 >= 2) {
                const Opt& a = o[hv[hv.size() - 2]];
                const Opt& b = o[hv.back()];
                // drop b if it lies on or above the segment a -> o[i]
                double lhs = (b.e - a.e) * (double)(o[i].s - a.s);
                double rhs = (o[i].e - a.e) * (double)(b.s - a.s);
                if (lhs >= rhs) hv.pop_back();
                else break;
            }
            hv.push_back(i);
        }
        hoff[c + 1] = (int64_t)hv.size();
    }
    auto eff_of = [&](int64_t c, int64_t h) {
        const Opt& a = cls(c)[hv[h - 1]];
        const Opt& b = cls(c)[hv[h]];
        return (a.e - b.e) / (double)(b.s - a.s);
    };
    std::vector<int>& pos = greedy_pos;  // current option position per class
    pos.assign(ncls, 0);
    int64_t cap = budget - min_total;
    lambda = 0.0;
    // The greedy takes the increments in the order of a heap merge of the
    // classes (largest efficiency first, ties to the smaller class).  When the
    // efficiencies fall along every class's hull -- always so in exact
    // arithmetic, rounding may break it -- that order is the sort by
    // (efficiency desc, class, hull position), and the increment where the
    // greedy stops (the first whose size no longer fits) is found by a
    // weighted selection in linear expected time.
    inc.clear();
    bool monotone = true;
    for (int64_t c = 0; c < ncls && monotone; ++c)
        for (int64_t h = hoff[c] + 1; h < hoff[c + 1]; ++h) {
            const double e = eff_of(c, h);
            if (h > hoff[c] + 1 && e > inc.back().eff) {
                monotone = false;
                break;
            }
            inc.push_back({e, cls(c)[hv[h]].s - cls(c)[hv[h - 1]].s, c, h});
        }
    if (monotone) {
        auto before = [](const Inc& x, const Inc& y) {
            if (x.eff != y.eff) return x.eff > y.eff;
            if (x.c != y.c) return x.c < y.c;
            return x.h < y.h;
        };
        // Invariant: the increments ordered before [lo, hi) are taken (their
        // sizes are off cap), those after it are not.
        size_t lo = 0, hi = inc.size();
        bool stop = false;
        Inc split{};
        while (lo < hi) {
            const size_t m = lo + (hi - lo) / 2, l = hi - 1;  // median of three as the pivot
            size_t piv = m;
            if (before(inc[lo], inc[m]) != before(inc[lo], inc[l])) piv = lo;
            else if (before(inc[l], inc[m]) != before(inc[l], inc[lo])) piv = l;
            std::swap(inc[lo], inc[piv]);
            const Inc p = inc[lo];
            size_t q = lo + 1;
            int64_t w = 0;  // size of the increments before the pivot
            for (size_t i = lo + 1; i < hi; ++i)
                if (before(inc[i], p)) {
                    w += inc[i].ds;
                    std::swap(inc[i], inc[q++]);
                }
            if (w > cap) {  // the stop lies before the pivot
                hi = q;
                lo = lo + 1;
            } else if (p.ds > cap - w) {  // the pivot is the stop
                cap -= w;
                split = p;
                stop = true;
                break;
            } else {
                cap -= w + p.ds;
                lo = q;
            }
        }
        // each class's taken increments are a prefix of its hull
        for (int64_t c = 0; c < ncls; ++c) {
            int64_t h = hoff[c] + 1;
            for (; h < hoff[c + 1]; ++h)
                if (stop && !before(Inc{eff_of(c, h), 0, c, h}, split)) break;
            pos[c] = hv[h - 1];
        }
        if (stop) lambda = split.eff;
    } else {
        // max-heap on (eff, then smaller class first)
        auto later = [](const Head& x, const Head& y) {
            if (x.eff != y.eff) return x.eff < y.eff;
            return x.c > y.c;
        };
        heap.clear();
        heap.reserve((size_t)ncls);
        for (int64_t c = 0; c < ncls; ++c)
            if (hoff[c + 1] - hoff[c] >= 2) heap.push_back({eff_of(c, hoff[c] + 1), c, hoff[c] + 1});
        std::make_heap(heap.begin(), heap.end(), later);
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), later);
            const Head hd = heap.back();
            heap.pop_back();
            const int from = hv[hd.h - 1], to = hv[hd.h];
            const int64_t ds = cls(hd.c)[to].s - cls(hd.c)[from].s;
            if (ds > cap) {
                lambda = hd.eff;
                break;
            }
            cap -= ds;
            pos[hd.c] = to;
            if (hd.h + 1 < hoff[hd.c + 1]) {
                heap.push_back({eff_of(hd.c, hd.h + 1), hd.c, hd.h + 1});
                std::push_heap(heap.begin(), heap.end(), later);
            }
        }
    }
    greedy_cap = cap;

    // ---- 3. Lagrangian bound, reduced costs, Lagrangian-best option per class
    mlam.assign(ncls, 0.0);
    lagbest.assign(ncls, 0);
    LB0 = -lambda * (double)budget;
    double scale = 0.0;
    for (int64_t c = 0; c < ncls; ++c) {
        double m = kInf;
        for (int i = 0; i < (int)cls(c).size(); ++i) {
            double v = cls(c)[i].e + lambda * (double)cls(c)[i].s;
            if (v < m) {  // options are sorted by size: ties keep the smaller size
                m = v;
                lagbest[c] = i;
            }
        }
        mlam[c] = m;
        LB0 += m;
        scale = std::max(scale, std::fabs(m));
    }
    // slack for the rounding of bounds (UB is close to LB0, so it adds nothing)
    tol = 1e-9 * (scale + std::fabs(LB0) + std::fabs(lambda * (double)budget)) + 1e-300;
    return MGS_OK;
    }

    // Phase 2, before an exact solve: the incumbent, the reduced costs and
    // the order of the classes by their cheapest alternative.
    void prepare_solve() {
    if (solve_ready || trivial) return;
    int64_t cap = greedy_cap;
    // incumbent: greedy solution improved by single-class moves
    inc_pos = greedy_pos;
    {
        bool improved = true;
        int rounds = 0;
        while (improved && rounds++ < 8) {
            improved = false;
            for (int64_t c = 0; c < ncls; ++c) {
                const auto& o = cls(c);
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
    UB = 0.0;
    for (int64_t c = 0; c < ncls; ++c) UB += cls(c)[inc_pos[c]].e;
    // smallest reduced cost of any other option of the class
    rcmin.assign(ncls, kInf);
    for (int64_t c = 0; c < ncls; ++c)
        for (int i = 0; i < (int)cls(c).size(); ++i)
            if (i != lagbest[c])
                rcmin[c] = std::min(rcmin[c], cls(c)[i].e + lambda * (double)cls(c)[i].s - mlam[c]);
    order.resize(ncls);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        if (rcmin[a] != rcmin[b]) return rcmin[a] < rcmin[b];
        return a < b;
    });
    solve_ready = true;
    }

    int exact(uint8_t* choice, double* obj, int64_t* used) {
        prepare_solve();  // (no-op when done already or trivial)
        if (trivial) {
            for (int64_t c = 0; c < ncls; ++c) choice[c] = (uint8_t)cls(c).back().j;
        } else {
            int rc = MGS_ELIMIT;
            for (const auto& sc : kSchedules) {
                rc = expand(choice, sc.beam, sc.k0, sc.exact_max);
                if (rc != MGS_ELIMIT) break;
            }
            if (rc) return rc;
        }
        double o = 0.0;
        int64_t u = 0;
        for (int64_t c = 0; c < ncls; ++c) {
            const Opt& x = opt_j(c, choice[c]);
            o += x.e;
            u += x.s;
        }
        *obj = o;
        *used = u;
        return MGS_OK;
    }

    int expand(uint8_t* choice, size_t beam, size_t k0, size_t exact_max) {
    // ---- 4. expanding core: DP over the classes whose alternatives are
    // cheapest in reduced cost improves the incumbent, which shrinks the gap;
    // once every class that can still change (rcmin <= gap) fits in the core,
    // one exact DP over exactly those classes finishes.
    size_t K = k0;
    for (;;) {
        const double gap = UB - LB0 + tol;
        std::vector<int64_t> need;
        for (int64_t c : order) {
            if (rcmin[c] > gap) break;
            need.push_back(c);
        }
        const bool final_pass = need.size() <= K;
        if (final_pass && need.size() > exact_max) return MGS_ELIMIT;  // the next schedule first
        std::vector<int64_t> core = final_pass ? need : std::vector<int64_t>(order.begin(), order.begin() + K);
        if (final_pass) std::sort(core.begin(), core.end());  // index order for the tie rule
        std::vector<char> in_core(ncls, 0);
        for (int64_t c : core) in_core[c] = 1;
        double e_fixed = 0.0;
        int64_t s_fixed = 0;
        for (int64_t c = 0; c < ncls; ++c)
            if (!in_core[c]) {
                e_fixed += cls(c)[lagbest[c]].e;
                s_fixed += cls(c)[lagbest[c]].s;
            }
        std::vector<std::vector<Opt>> opts(core.size());
        for (size_t i = 0; i < core.size(); ++i)
            for (const Opt& x : cls(core[i]))
                if (x.e + lambda * (double)x.s - mlam[core[i]] <= gap) opts[i].push_back(x);
        std::vector<int16_t> pick;
        double zb = 0.0;
        int rc = core_dp(opts, e_fixed, budget - s_fixed, lambda, UB, tol,
                         final_pass ? 0 : beam, pick);
        if (rc == MGS_ELIMIT) return rc;
        if (final_pass) {
            if (rc != MGS_OK) return MGS_EINFEASIBLE;  // (cannot happen: the incumbent is a state)
            for (int64_t c = 0; c < ncls; ++c)
                if (!in_core[c]) choice[c] = (uint8_t)cls(c)[lagbest[c]].j;
            for (size_t i = 0; i < core.size(); ++i) choice[core[i]] = (uint8_t)pick[i];
            break;
        }
        if (rc == MGS_OK) {
            zb = e_fixed;
            for (size_t i = 0; i < core.size(); ++i) zb += opt_j(core[i], pick[i]).e;
            if (zb < UB) UB = zb;
        } else if (K >= kWideAfter && exact_max != kNoLimit) {
            // this beam found nothing better over a core of this size: a wider
            // beam over a small core is the cheaper way on (the next schedule)
            return MGS_ELIMIT;
        }
        K *= 4;
    }
    return MGS_OK;
    }
};

int solve(const double* err, const int64_t* size, int64_t ncls, int nopt, int64_t budget,
          uint8_t* choice, double* obj, int64_t* used) {
    Mckp m(err, size, ncls, nopt, budget);
    int rc = m.prepare();
    if (rc) return rc;
    return m.exact(choice, obj, used);
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

// The ILP instance of ratio t from a sweep's host tables (layout of
// mgs_quant_sweep): loss and entropy bits per (class, option), classes
// channel-major then group, and each class's element count.  False if a
// loss is not finite.
static bool ratio_instance(const mgs_sweep_desc* d, const double* h_err, const double* h_bits, int t,
                           int64_t gmaxn, std::vector<double>& E, std::vector<double>& B,
                           std::vector<int64_t>& n) {
    const int C = d->C, G = d->G, nb = d->nb;
    const int64_t k = d->h_k[t];
    const int64_t ng = (k + G - 1) / G;
    const int64_t ncls = (int64_t)C * ng;
    E.resize(ncls * nb);
    B.resize(ncls * nb);
    n.resize(ncls);
    for (int c = 0; c < C; ++c)
        for (int64_t g = 0; g < ng; ++g) {
            const int64_t cls = (int64_t)c * ng + g;
            const int64_t slot = ((int64_t)t * C + c) * gmaxn + g;
            n[cls] = std::min<int64_t>(G, k - g * G);
            for (int i = 0; i < nb; ++i) {
                E[cls * nb + i] = h_err[slot * nb + i];
                B[cls * nb + i] = h_bits[slot * nb + i];
            }
        }
    for (double v : E)
        if (!std::isfinite(v)) return false;
    return true;
}

namespace mgs {
// The search over one sweep's tables.  `wait`, when not NULL, tells whether
// ratio t's entries are on the host yet (the tables may still be on their way):
// wait(ctx, t, 1) returns once they are, wait(ctx, t, 0) returns at once, 1
// while they are not; MGS_OK means they are, anything else is the search's
// error.
int search_tables(const mgs_sweep_desc* d, const double* h_err, const double* h_bits, int64_t budget_bits,
                  int32_t size_mode, int32_t threads, int32_t flags, int32_t* h_best_t, uint8_t* h_best_bits,
                  double* h_obj, int64_t* h_used, int32_t* h_status, int (*wait)(void*, int, int), void* wait_ctx) {
    if (!d || !d->h_k || !d->h_bits || !h_err || !h_bits || !h_best_t || !h_best_bits || !h_obj ||
        !h_used)
        return MGS_EINVAL;
    if (d->C < 1 || d->T < 1 || d->T > MGS_MAX_RATIOS || d->G < 1 || d->nb < 1 ||
        d->nb > MGS_MAX_BITS || (size_mode != 0 && size_mode != 1))
        return MGS_EINVAL;
    const int C = d->C, T = d->T, G = d->G, nb = d->nb;
    int64_t kmax = 0;
    for (int t = 0; t < T; ++t) {
        if (d->h_k[t] < 0) return MGS_EINVAL;
        kmax = std::max(kmax, d->h_k[t]);
    }
    const int64_t gmaxn = (kmax + G - 1) / G;
    // ratio t's entries are on the host (waited for once, by any thread)
    std::unique_ptr<std::atomic<int>[]> landed(new std::atomic<int>[T]);
    for (int t = 0; t < T; ++t) landed[t].store(wait ? 0 : 1, std::memory_order_relaxed);
    std::atomic<int> wait_rc{MGS_OK};
    auto wait_ratio = [&](int t) {
        if (landed[t].load(std::memory_order_acquire)) return;
        const int rc = wait(wait_ctx, t, 1);
        if (rc != MGS_OK) wait_rc.store(rc);
        landed[t].store(1, std::memory_order_release);
    };
    // without blocking: true once ratio t is on the host (or failed)
    auto poll_ratio = [&](int t) {
        if (landed[t].load(std::memory_order_acquire)) return true;
        const int rc = wait(wait_ctx, t, 0);
        if (rc == 1) return false;
        if (rc != MGS_OK) wait_rc.store(rc);
        landed[t].store(1, std::memory_order_release);
        return true;
    };
    int b8 = -1;
    for (int i = 0; i < nb; ++i)
        if (d->h_bits[i] == 8) b8 = i;
    const int nthr = threads > 0 ? threads : omp_get_max_threads();
    std::vector<int> st(T, MGS_OK), state(T, MGS_SEARCH_SOLVED);
    std::vector<double> lb(T, 0.0), lbtol(T, 0.0);
    // The options of class (channel c, group g) of ratio t straight from the
    // tables: loss row, and size by the rule of mgs_size_table.  False on a
    // loss that is not finite or (entropy sizes) a size that is not finite
    // and nonnegative.
    auto filler = [&](int t) -> Mckp::Fill {
        const int64_t k = d->h_k[t], ng = (k + G - 1) / G;
        return [=](int64_t cls, Opt* o) {
            const int64_t c = cls / ng, g = cls - c * ng;
            const int64_t slot = ((int64_t)t * C + c) * gmaxn + g;
            const double* e = h_err + slot * nb;
            const double* b = h_bits + slot * nb;
            const int64_t n = std::min<int64_t>(G, k - g * G);
            bool ok = true;
            for (int i = 0; i < nb; ++i) {
                ok = ok && std::isfinite(e[i]) && (size_mode == 1 || (std::isfinite(b[i]) && b[i] >= 0));
                o[i] = {e[i], size_mode == 0 ? (ok ? (int64_t)std::ceil(b[i]) : 0) + kMetaBits
                                             : n * (int64_t)d->h_bits[i] + kMetaBits, i};
            }
            return ok;
        };
    };

    // ---- per ratio: checks of the tables, the doubled-8-bit test, LP bound.
    // Largest ratios first (the cost grows with k); each thread bounds its
    // ratios in one long-lived instance, so that repeated searches reuse its
    // arrays.
    std::vector<int> by_k(T);
    std::iota(by_k.begin(), by_k.end(), 0);
    std::stable_sort(by_k.begin(), by_k.end(), [&](int a, int b) { return d->h_k[a] > d->h_k[b]; });
    // The smallest ratio that passes the doubled-8-bit test usually has the
    // least bound, so it is solved at once, beside the other bounds; its
    // result is used only where the ratio is solved anyway.
    int t_spec = -1;
    for (int i = T - 1; i >= 0 && t_spec < 0; --i) {
        const int t = by_k[i];
        wait_ratio(t);
        const int64_t k = d->h_k[t], ng = (k + G - 1) / G;
        int64_t s8 = 0;
        bool ok = true;
        for (int c = 0; c < C && ok; ++c)
            for (int64_t g = 0; g < ng; ++g) {
                const int64_t n = std::min<int64_t>(G, k - g * G);
                if (b8 < 0 || size_mode == 1) {
                    s8 += n * 8 + kMetaBits;
                } else {
                    const double b = h_bits[(((int64_t)t * C + c) * gmaxn + g) * nb + b8];
                    if (!(std::isfinite(b) && b >= 0)) {
                        ok = false;
                        break;
                    }
                    s8 += (int64_t)std::ceil(b) + kMetaBits;
                }
            }
        if (!ok) break;  // the pass below reports it
        if (ng > 0 && 2 * s8 >= budget_bits) t_spec = t;
    }
    std::vector<int> items;
    if (t_spec >= 0) items.push_back(t_spec);
    for (int t : by_k)
        if (t != t_spec) items.push_back(t);
    std::vector<std::vector<uint8_t>> choice(T);
    int spec_rc = MGS_EINVAL;  // the speculative solve: status, loss, size
    double spec_obj = 0;
    int64_t spec_used = 0;
    // The speculative ratio's LP and greedy incumbent come first: its
    // multiplier gives every other ratio a bound in one pass over the options
    // (the Lagrangian bound at a fixed multiplier, below the LP bound), and
    // a ratio whose bound exceeds the incumbent's loss cannot win or tie (its
    // optimum is at least that bound, the incumbent's loss at least the best
    // optimum): it is not solved, and needs no LP bound of its own.
    Mckp spec_m;
    int spec_prep = MGS_EINVAL;
    double lam_spec = 0.0, ub_spec = kInf;
    if (t_spec >= 0) {
        const int64_t ncls = (int64_t)C * ((d->h_k[t_spec] + G - 1) / G);
        spec_m.rebind(filler(t_spec), ncls, nb, budget_bits);
        spec_prep = spec_m.prepare_bound();
        if (spec_prep == MGS_OK && !(flags & MGS_SEARCH_ALL)) {  // (every ratio solved: nothing to prune)
            spec_m.prepare_solve();
            lam_spec = spec_m.lambda;
            ub_spec = spec_m.trivial ? spec_m.lower_bound() : spec_m.UB;
        }
    }
    // The one-pass bound of ratio t at multiplier lam: sum over classes of
    // min_i (loss_i + lam size_i), minus lam times the budget; also the
    // smallest total size.  False on an invalid option.
    auto fixed_bound = [&](int t, double lam, double* lbw, double* tolw, int64_t* min_total) {
        const int64_t ncls = (int64_t)C * ((d->h_k[t] + G - 1) / G);
        const Mckp::Fill f = filler(t);
        Opt o[MGS_MAX_BITS];
        double sum = 0.0, scale = 0.0;
        int64_t mt = 0;
        for (int64_t cls = 0; cls < ncls; ++cls) {
            if (!f(cls, o)) return false;
            double m = kInf;
            int64_t smin = o[0].s;
            for (int i = 0; i < nb; ++i) {
                m = std::min(m, o[i].e + lam * (double)o[i].s);
                smin = std::min(smin, o[i].s);
            }
            sum += m;
            scale = std::max(scale, std::fabs(m));
            mt += smin;
        }
        *lbw = sum - lam * (double)budget_bits;
        *tolw = 1e-9 * (scale + std::fabs(*lbw) + std::fabs(lam * (double)budget_bits)) + 1e-300;
        *min_total = mt;
        return true;
    };
    // per ratio: the checks, the doubled-8-bit test and the LP bound (the
    // speculative ratio is solved exactly as well)
    auto process = [&](int t) {
        h_obj[t] = std::numeric_limits<double>::quiet_NaN();
        h_used[t] = 0;
        const int64_t k = d->h_k[t];
        const int64_t ng = (k + G - 1) / G;
        const int64_t ncls = (int64_t)C * ng;
        if (ncls == 0) {
            state[t] = MGS_SEARCH_SKIPPED;
            return;
        }
        // the all-8-bit size from the 8-bit column alone; every value of the
        // ratio is checked by the bound's pass over the options, or by a pass
        // of its own when the ratio is skipped
        int64_t s8 = 0;
        bool ok = true;
        for (int c = 0; c < C; ++c)
            for (int64_t g = 0; g < ng; ++g) {
                const int64_t n = std::min<int64_t>(G, k - g * G);
                if (b8 < 0 || size_mode == 1) {
                    s8 += n * 8 + kMetaBits;
                } else {
                    const double b = h_bits[(((int64_t)t * C + c) * gmaxn + g) * nb + b8];
                    if (std::isfinite(b) && b >= 0) s8 += (int64_t)std::ceil(b) + kMetaBits;
                    else ok = false;
                }
            }
        if (ok && 2 * s8 < budget_bits) {
            Opt o[MGS_MAX_BITS];
            const Mckp::Fill f = filler(t);
            for (int64_t cls = 0; cls < ncls && ok; ++cls) ok = f(cls, o);
            if (ok) {
                state[t] = MGS_SEARCH_SKIPPED;
                return;
            }
        }
        if (!ok) {
            st[t] = MGS_EINVAL;
            return;
        }
        if (t == t_spec) {
            const int rc = spec_prep;
            if (rc == MGS_EINFEASIBLE) state[t] = MGS_SEARCH_INFEASIBLE;
            else st[t] = rc;
            lb[t] = spec_m.lower_bound();
            lbtol[t] = spec_m.tol;
            if (rc == MGS_OK) {
                choice[t].resize(ncls);
                spec_rc = spec_m.exact(choice[t].data(), &spec_obj, &spec_used);
            }
            return;
        }
        if (ub_spec < kInf) {
            double lbw = 0.0, tolw = 0.0;
            int64_t mt = 0;
            if (!fixed_bound(t, lam_spec, &lbw, &tolw, &mt)) {
                st[t] = MGS_EINVAL;
                return;
            }
            if (mt > budget_bits) {
                state[t] = MGS_SEARCH_INFEASIBLE;
                return;
            }
            if (lbw - tolw > ub_spec + 1e-12 * std::fabs(ub_spec)) {
                state[t] = MGS_SEARCH_PRUNED;
                lb[t] = lbw;
                return;
            }
        }
        static thread_local Mckp wk;
        wk.rebind(filler(t), ncls, nb, budget_bits);
        const int rc = wk.prepare_bound();
        if (rc == MGS_EINFEASIBLE) state[t] = MGS_SEARCH_INFEASIBLE;
        else st[t] = rc;
        lb[t] = wk.lower_bound();
        lbtol[t] = wk.tol;
    };
    if (!wait) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
        for (int i = 0; i < T; ++i) process(items[i]);
    } else {
        // tables still arriving: the speculative ratio (already on the host,
        // the pick above waited for it) on a thread of its own at once; one
        // thread polls the other ratios and hands each to the pool as it lands
        std::thread spec;
        int first = 0;
        if (t_spec >= 0) {
            spec = std::thread([&] { process(t_spec); });
            first = 1;
        }
        std::vector<int> pending(items.begin() + first, items.end());
#pragma omp parallel num_threads(nthr)
#pragma omp single
        while (!pending.empty() && wait_rc.load() == MGS_OK) {
            bool any = false;
            for (size_t j = 0; j < pending.size();) {
                const int t = pending[j];
                if (!poll_ratio(t)) {
                    ++j;
                    continue;
                }
#pragma omp task firstprivate(t)
                process(t);
                pending[j] = pending.back();
                pending.pop_back();
                any = true;
            }
            if (!any) std::this_thread::yield();
        }
        if (spec.joinable()) spec.join();
    }
    if (wait_rc.load() != MGS_OK) return wait_rc.load();
    for (int t = 0; t < T; ++t)
        if (st[t] != MGS_OK) return st[t];
    // ---- exact solves: the ratio of least lower bound first, then (in
    // parallel) every ratio whose bound does not exceed that optimum -- the
    // others cannot win (or tie) -- unless every ratio is asked for.  A solved
    // ratio builds its instance again (the same bound) and keeps its choice.
    std::vector<int> cand;
    for (int t = 0; t < T; ++t)
        if (state[t] == MGS_SEARCH_SOLVED) cand.push_back(t);
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return lb[a] < lb[b]; });
    auto solve_one = [&](int t) {
        const int64_t ncls = (int64_t)C * ((d->h_k[t] + G - 1) / G);
        int rc = MGS_OK;
        double o = 0;
        int64_t u = 0;
        if (t == t_spec) {
            rc = spec_rc;
            o = spec_obj;
            u = spec_used;
        } else {
            Mckp m(filler(t), ncls, nb, budget_bits);
            choice[t].resize(ncls);
            rc = m.prepare_bound();
            if (rc == MGS_OK) rc = m.exact(choice[t].data(), &o, &u);
        }
        st[t] = rc;
        if (rc == MGS_OK) {
            h_obj[t] = o;
            h_used[t] = u;
        }
    };
    std::vector<int> todo;
    if (flags & MGS_SEARCH_ALL) {
        todo = cand;
    } else if (!cand.empty()) {
        solve_one(cand[0]);
        if (st[cand[0]] != MGS_OK) return st[cand[0]];
        const double best0 = h_obj[cand[0]];
        for (size_t i = 1; i < cand.size(); ++i) {
            const int t = cand[i];
            if (lb[t] <= best0 + lbtol[t] + 1e-12 * std::fabs(best0))
                todo.push_back(t);
            else
                state[t] = MGS_SEARCH_PRUNED;
        }
    }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int i = 0; i < (int)todo.size(); ++i) solve_one(todo[i]);
    for (int t = 0; t < T; ++t)
        if (st[t] != MGS_OK) return st[t];
    if (h_status)
        for (int t = 0; t < T; ++t) h_status[t] = state[t];
    int best = -1;
    for (int t = 0; t < T; ++t) {
        if (state[t] != MGS_SEARCH_SOLVED) continue;
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

}  // namespace mgs

extern "C" int mgs_search(const mgs_sweep_desc* d, const double* h_err, const double* h_bits,
                          int64_t budget_bits, int32_t size_mode, int32_t threads, int32_t flags,
                          int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_used,
                          int32_t* h_status) {
    return mgs::search_tables(d, h_err, h_bits, budget_bits, size_mode, threads, flags, h_best_t, h_best_bits,
                              h_obj, h_used, h_status, nullptr, nullptr);
}

// ------------------------------------------------------------- hierarchical solver
// Paper, section "Hierarchical Solver": first the channel-level bit-widths
// Q_c (one option per channel, shared by all of its groups), then each
// channel's budget S_c = S_T * Q_c / sum_c Q_c and, per channel, the
// group-level ILP within S_c.  Both steps use the exact solver above.
extern "C" int mgs_ilp_hierarchical(const double* h_err, const int64_t* h_size, int32_t C, int64_t ng,
                                    int32_t nopt, const uint8_t* h_bitlist, int64_t budget,
                                    uint8_t* h_choice, double* h_obj, int64_t* h_used,
                                    uint8_t* h_chan_bits, int64_t* h_chan_budget) {
    if (C < 1 || ng < 1 || nopt < 1 || nopt > 255 || budget < 0 || !h_err || !h_size || !h_bitlist ||
        !h_choice || !h_obj || !h_used)
        return MGS_EINVAL;
    const int64_t ncls = (int64_t)C * ng;
    for (int64_t i = 0; i < ncls * nopt; ++i)
        if (!std::isfinite(h_err[i]) || h_size[i] < 0) return MGS_EINVAL;
    for (int j = 0; j < nopt; ++j)
        if (h_bitlist[j] < 1) return MGS_EINVAL;
    // step 1: a channel's option is every one of its groups at that option;
    // its loss and size are the sums over the groups (in group order)
    std::vector<double> ec((size_t)C * nopt, 0.0);
    std::vector<int64_t> sc((size_t)C * nopt, 0);
    for (int c = 0; c < C; ++c)
        for (int64_t g = 0; g < ng; ++g)
            for (int j = 0; j < nopt; ++j) {
                ec[(size_t)c * nopt + j] += h_err[((int64_t)c * ng + g) * nopt + j];
                sc[(size_t)c * nopt + j] += h_size[((int64_t)c * ng + g) * nopt + j];
            }
    std::vector<uint8_t> qc((size_t)C);
    double o = 0.0;
    int64_t u = 0;
    int rc = solve(ec.data(), sc.data(), C, nopt, budget, qc.data(), &o, &u);
    if (rc) return rc;
    // step 2: the channel shares of the budget, then each channel alone
    int64_t qsum = 0;
    for (int c = 0; c < C; ++c) qsum += h_bitlist[qc[c]];
    double obj = 0.0;
    int64_t used = 0;
    for (int c = 0; c < C; ++c) {
        const int64_t share = (int64_t)((__int128)budget * h_bitlist[qc[c]] / qsum);
        if (h_chan_bits) h_chan_bits[c] = h_bitlist[qc[c]];
        if (h_chan_budget) h_chan_budget[c] = share;
        rc = solve(h_err + (int64_t)c * ng * nopt, h_size + (int64_t)c * ng * nopt, ng, nopt, share,
                   h_choice + (int64_t)c * ng, &o, &u);
        if (rc) return rc;  // MGS_EINFEASIBLE: the share cannot hold the channel's cheapest allocation
        obj += o;
        used += u;
    }
    *h_obj = obj;
    *h_used = used;
    return MGS_OK;
}

// ------------------------------------------------------- calibrated search (Algorithm 1)
// Paper: Algorithm 1 "Hyperparameter Optimization" with the linear size
// estimator of equation "size_estim" (n * b bits per group plus its 72
// metadata bits, plus the calibration term S_delta).  Per ratio: the all-8-bit
// configuration gives the first measured size S_a; a ratio whose doubled S_a
// is below the budget is skipped; then repeatedly S_delta = S_a - (linear
// estimate of the current allocation), the exact ILP with linear sizes under
// the budget S_T - S_delta gives the next allocation, and its measured size
// S_a (the entropy table: ceil(bits) + 72 per group) ends the loop once
// |S_a - S_T| < tol * S_T.  Among converged ratios the smallest loss wins
// (ties: larger k, then larger index).
extern "C" int mgs_search_calibrated(const mgs_sweep_desc* d, const double* h_err, const double* h_bits,
                                     int64_t budget_bits, int32_t tol_ppm, int32_t max_iter,
                                     int32_t threads, int32_t* h_best_t, uint8_t* h_best_bits,
                                     double* h_obj, int64_t* h_actual, int32_t* h_iters,
                                     int32_t* h_status) {
    if (!d || !d->h_k || !d->h_bits || !h_err || !h_bits || !h_best_t || !h_best_bits || !h_obj ||
        !h_actual || !h_iters)
        return MGS_EINVAL;
    if (d->C < 1 || d->T < 1 || d->T > MGS_MAX_RATIOS || d->G < 1 || d->nb < 1 ||
        d->nb > MGS_MAX_BITS || budget_bits < 1 || tol_ppm < 0 || tol_ppm > 1000000 || max_iter < 1)
        return MGS_EINVAL;
    const int C = d->C, T = d->T, G = d->G, nb = d->nb;
    int64_t kmax = 0;
    for (int t = 0; t < T; ++t) {
        if (d->h_k[t] < 0) return MGS_EINVAL;
        kmax = std::max(kmax, d->h_k[t]);
    }
    const int64_t gmaxn = (kmax + G - 1) / G;
    int b8 = -1;
    for (int i = 0; i < nb; ++i)
        if (d->h_bits[i] == 8) b8 = i;
    const int nthr = threads > 0 ? threads : omp_get_max_threads();
    std::vector<int> st(T, MGS_OK), state(T, MGS_SEARCH_UNCONVERGED);
    std::vector<std::vector<uint8_t>> choice(T);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr)
    for (int t = 0; t < T; ++t) {
        h_obj[t] = std::numeric_limits<double>::quiet_NaN();
        h_actual[t] = 0;
        h_iters[t] = 0;
        const int64_t ng = (d->h_k[t] + G - 1) / G;
        const int64_t ncls = (int64_t)C * ng;
        if (ncls == 0) {
            state[t] = MGS_SEARCH_SKIPPED;
            continue;
        }
        std::vector<double> E, B;
        std::vector<int64_t> n;
        if (!ratio_instance(d, h_err, h_bits, t, gmaxn, E, B, n)) {
            st[t] = MGS_EINVAL;
            continue;
        }
        std::vector<int64_t> act(ncls * nb), lin(ncls * nb);
        int rc = mgs_size_table(B.data(), n.data(), ncls, nb, d->h_bits, 0, act.data());
        if (!rc) rc = mgs_size_table(B.data(), n.data(), ncls, nb, d->h_bits, 1, lin.data());
        if (rc) {
            st[t] = rc;
            continue;
        }
        int64_t sa = 0, est = 0;  // measured and estimated size of the all-8-bit start
        for (int64_t cls = 0; cls < ncls; ++cls) {
            sa += (b8 >= 0) ? act[cls * nb + b8] : n[cls] * 8 + kMetaBits;
            est += n[cls] * 8 + kMetaBits;
        }
        h_actual[t] = sa;
        if (2 * sa < budget_bits) {
            state[t] = MGS_SEARCH_SKIPPED;
            continue;
        }
        choice[t].resize(ncls);
        for (int it = 1; it <= max_iter; ++it) {
            const int64_t delta = sa - est;
            double o = 0.0;
            int64_t u = 0;
            rc = solve(E.data(), lin.data(), ncls, nb, budget_bits - delta, choice[t].data(), &o, &u);
            if (rc == MGS_EINFEASIBLE) {
                state[t] = MGS_SEARCH_INFEASIBLE;
                break;
            }
            if (rc) {
                st[t] = rc;
                break;
            }
            sa = 0;
            for (int64_t cls = 0; cls < ncls; ++cls) sa += act[cls * nb + choice[t][cls]];
            est = u;
            h_obj[t] = o;
            h_actual[t] = sa;
            h_iters[t] = it;
            const int64_t dev = sa > budget_bits ? sa - budget_bits : budget_bits - sa;
            if (dev * 1000000 < (int64_t)tol_ppm * budget_bits) {
                state[t] = MGS_SEARCH_SOLVED;
                break;
            }
        }
    }
    for (int t = 0; t < T; ++t)
        if (st[t] != MGS_OK) return st[t];
    if (h_status)
        for (int t = 0; t < T; ++t) h_status[t] = state[t];
    int best = -1;
    for (int t = 0; t < T; ++t) {
        if (state[t] != MGS_SEARCH_SOLVED) continue;
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
