"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: the expected values are worked
by hand from the quantizer and entropy definitions, closed forms, invariants
that hold for any input, brute force over tiny inputs, or library routines
(scipy's entropy and MILP solver, Python's sort).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def one_group(orc, x, b, w=None):
    """Run one group through every oracle entry point; return codes, xhat, err, bits, hist."""
    x = np.asarray(x, dtype=np.float32)
    n = x.size
    w = np.ones(n, np.float32) if w is None else np.asarray(w, np.float32)
    attr = x.reshape(1, n)
    kept = np.arange(n, dtype=np.int32)
    k = np.array([n], np.int64)
    sw = orc.quant_sweep(attr, w, kept, k, n, [b], want_hist=True)
    codes, mn, mx = orc.quantize(attr, kept, n, np.array([[b]], np.uint8))
    xhat = orc.dequantize(codes, n, np.array([[b]], np.uint8), mn, mx)
    return codes[0], xhat[0], sw["err"][0, 0, 0, 0], sw["bits"][0, 0, 0, 0], sw["hist"][0, 0, 0]


# ---------------------------------------------------------------- quantizer
def test_hand_cases(orc):
    cases = json.load(open(os.path.join(HERE, "golden", "quantizer_hand_cases.json")))["cases"]
    for c in cases:
        codes, xhat, err, bits, hist = one_group(orc, c["x"], c["b"], c.get("w"))
        assert codes.tolist() == c["codes"], c
        assert np.array_equal(xhat, np.asarray(c["xhat"], np.float32)), c
        assert err == c["err"], c
        assert bits == pytest.approx(c["bits"], rel=1e-14, abs=1e-14), c
        assert hist.sum() == len(c["x"])


@pytest.mark.parametrize("b", [1, 2, 3, 5, 8, 12, 16])
def test_lattice_closed_form(orc, b):
    """Values on the quantization lattice {0, S, ..., 2^b S} (for large b a random
    subset keeping both ends): every element but the top one is reconstructed
    exactly and the top one is clamped one step down, so err = S^2 exactly."""
    S = 2.0 ** -3
    rng = np.random.default_rng(b)
    if b <= 12:
        m = np.arange(2 ** b + 1, dtype=np.float64)
    else:
        mid = rng.choice(np.arange(1, 2 ** b), 3000, replace=False)
        m = np.sort(np.concatenate([[0, 2 ** b], mid])).astype(np.float64)
    x = (m * S).astype(np.float32)
    codes, xhat, err, bits, hist = one_group(orc, x, b)
    want = np.minimum(m, 2 ** b - 1).astype(np.uint16)
    assert np.array_equal(codes, want)
    assert np.array_equal(xhat[:-1], x[:-1])
    assert xhat[-1] == np.float32((2 ** b - 1) * S)
    assert err == S * S
    n = x.size
    if b <= 12:  # every code once, the last one twice
        assert bits == pytest.approx((2 ** b - 1) * math.log2(n) + 2 * math.log2(n / 2), rel=1e-13)
    else:  # all codes distinct (2^b - 1 drawn or not): n - 1 singletons or n distinct
        two = (m == 2 ** b - 1).any()
        want_bits = (n - 2) * math.log2(n) + 2 * math.log2(n / 2) if two else n * math.log2(n)
        assert bits == pytest.approx(want_bits, rel=1e-13)


@pytest.mark.parametrize("b", [1, 4, 9, 16])
def test_shifted_lattice_negative_zero_point(orc, b):
    """Lattice shifted to [1, 1 + 2^b S]: Z = round(2^b - max/S) = -1/S exactly, so the
    codes are unchanged by the shift (a dropped or sign-flipped Z fails this)."""
    S = 2.0 ** -2
    m = np.arange(2 ** b + 1, dtype=np.float64) if b < 16 else \
        np.concatenate([np.arange(0, 2 ** b, 37), [2 ** b]]).astype(np.float64)
    x = (1.0 + m * S).astype(np.float32)
    codes, xhat, err, _, _ = one_group(orc, x, b)
    assert np.array_equal(codes, np.minimum(m, 2 ** b - 1).astype(np.uint16))
    assert np.array_equal(xhat[:-1], x[:-1])
    assert err == S * S


def test_constant_and_tiny_groups(orc):
    for x in ([3.5], [-2.0, -2.0], [0.0, -0.0, 0.0]):
        for b in (1, 7, 16):
            codes, xhat, err, bits, hist = one_group(orc, x, b)
            assert (codes == 0).all() and err == 0.0 and bits == 0.0
            assert (xhat == np.float32(x[0])).all()
            assert hist[0] == len(x)


def random_group(rng, n):
    kind = rng.integers(0, 4)
    if kind == 0:
        x = rng.normal(0, 1, n)
    elif kind == 1:
        x = rng.laplace(0, 0.05, n)
    elif kind == 2:
        x = rng.normal(-4, 1, n) * 10.0 ** rng.integers(-20, 20)
    else:
        x = rng.integers(-5, 5, n) * 0.5 + 100.0
    return x.astype(np.float32), rng.lognormal(0, 2, n).astype(np.float32)


def test_invariants_random_groups(orc):
    """Codes in range, histogram sums to n, H <= b and H <= log2 n per value,
    reconstruction within half a step away from the top clamp and 1.5 steps at
    it, loss nonincreasing in b."""
    rng = np.random.default_rng(7)
    bl = list(range(1, 17))
    for trial in range(60):
        n = int(rng.integers(1, 700))
        x, w = random_group(rng, n)
        attr = x.reshape(1, n)
        kept = np.arange(n, dtype=np.int32)
        sw = orc.quant_sweep(attr, w, kept, np.array([n]), n, bl, want_hist=True)
        err = sw["err"][0, 0, 0]
        bits = sw["bits"][0, 0, 0]
        mn, mx = float(sw["gmin"][0, 0, 0]), float(sw["gmax"][0, 0, 0])
        assert mn == x.min() and mx == x.max()
        off = 0
        for i, b in enumerate(bl):
            h = sw["hist"][0, 0, 0, off:off + 2 ** b]
            off += 2 ** b
            assert h.sum() == n
            assert bits[i] <= b * n * (1 + 1e-12) + 1e-9
            assert bits[i] <= n * math.log2(n) * (1 + 1e-12) + 1e-9
            codes, gmn, gmx = orc.quantize(attr, kept, n, np.array([[b]], np.uint8))
            assert int(codes.max()) <= 2 ** b - 1
            assert np.array_equal(np.bincount(codes[0], minlength=2 ** b), h)
            xhat = orc.dequantize(codes, n, np.array([[b]], np.uint8), gmn, gmx)[0]
            R = np.float32(mx) - np.float32(mn)
            S = float(R / np.float32(2.0 ** b))
            if S == 0.0:
                assert err[i] == 0.0 or mn != mx
                continue
            slack = 2.0 ** -21 * (np.abs(x).astype(np.float64) + abs(mn) + abs(mx)) + 1e-300
            dev = np.abs(xhat.astype(np.float64) - x.astype(np.float64))
            assert (dev <= 1.5 * S + slack).all()
            interior = x.astype(np.float64) <= mn + (2 ** b - 2) * S
            assert (dev[interior] <= 0.5 * S + slack[interior]).all()
        # the loss never grows with more bits (exact in real arithmetic; tiny slack
        # for the rounding of t in FP32)
        for i in range(len(bl) - 1):
            assert err[i + 1] <= err[i] * (1 + 1e-6) + 1e-300, (trial, bl[i], err[i], err[i + 1])


def test_loss_exact_rational(orc):
    """The FP64 loss equals the exact rational sum of w (xhat - x)^2 over the FP32
    values to 1e-13 relative."""
    rng = np.random.default_rng(3)
    for trial in range(20):
        n = int(rng.integers(2, 200))
        x, w = random_group(rng, n)
        for b in (1, 3, 8, 16):
            codes, xhat, err, _, _ = one_group(orc, x, b, w)
            exact = sum(Fraction(float(wj)) * (Fraction(float(xh)) - Fraction(float(xj))) ** 2
                        for wj, xh, xj in zip(w, xhat, x))
            if exact == 0:
                assert err == 0.0
            else:
                assert abs(Fraction(err) - exact) <= Fraction(1, 10 ** 13) * exact


def test_entropy_matches_scipy(orc):
    """The size table equals n times scipy's base-2 entropy of the code histogram."""
    from scipy.stats import entropy
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(1, 3000))
        x, w = random_group(rng, n)
        bl = [1, 2, 5, 9, 16]
        sw = orc.quant_sweep(x.reshape(1, n), w, np.arange(n, dtype=np.int32), np.array([n]), n, bl,
                             want_hist=True)
        off = 0
        for i, b in enumerate(bl):
            h = sw["hist"][0, 0, 0, off:off + 2 ** b].astype(np.float64)
            off += 2 ** b
            want = n * entropy(h, base=2) if h.sum() > 0 else 0.0
            assert sw["bits"][0, 0, 0, i] == pytest.approx(want, rel=1e-12, abs=1e-9)


def test_uniform_histogram_entropy(orc):
    """Every code used equally often -> exactly n*b bits."""
    for b in (1, 2, 4, 8):
        reps = 3
        m = np.repeat(np.arange(2 ** b, dtype=np.float64), reps)
        x = np.append(m, 2 ** b).astype(np.float32)  # top element clamps onto the last code
        # drop one copy of the last code so every code appears exactly `reps` times
        x = np.delete(x, np.where(x == 2 ** b - 1)[0][0])
        _, _, _, bits, hist = one_group(orc, x, b)
        assert (hist == reps).all()
        assert bits == pytest.approx(x.size * b, rel=1e-14)


def test_groups_and_ratios_layout(orc):
    """Tables of several ratios / channels / ragged groups equal the one-group
    results of the same slices (the layout [t][c][g][b] and NaN padding)."""
    from paper_2604_26799_amd import synth
    attr, imp = synth.scene(3000, 11, seed=5)
    k = np.array([700, 3000, 1501], np.int64)
    kept = orc.prune_select(imp, k)
    G, bl = 256, [2, 5, 16]
    sw = orc.quant_sweep(attr, imp, kept, k, G, bl)
    gm = (3000 + G - 1) // G
    assert sw["err"].shape == (3, 11, gm, 3)
    offs = np.concatenate([[0], np.cumsum(k)])
    for t in range(3):
        J = kept[offs[t]:offs[t + 1]]
        ng = (k[t] + G - 1) // G
        assert np.isnan(sw["err"][t, :, ng:]).all()
        for c in (0, 3, 10):
            for g in (0, ng - 1):
                sl = J[g * G:(g + 1) * G]
                x = attr[c, sl]
                for i, b in enumerate(bl):
                    _, _, e, s, _ = one_group(orc, x, b, imp[sl])
                    assert sw["err"][t, c, g, i] == e and sw["bits"][t, c, g, i] == s


def test_nonfinite_rejected(orc):
    x = np.array([[0.0, np.inf, 1.0]], np.float32)
    with pytest.raises(orc.OracleError) as e:
        orc.quant_sweep(x, np.ones(3, np.float32), np.arange(3, dtype=np.int32), np.array([3]), 3, [4])
    assert e.value.code == orc.ENONFINITE


# ---------------------------------------------------------------- pruning
def test_prune_hand_ties(orc):
    imp = np.array([1, 3, 3, 2, 3], np.float32)
    kept = orc.prune_select(imp, [2, 3, 4, 0, 5])
    assert kept.tolist() == [1, 2] + [1, 2, 4] + [1, 2, 3, 4] + [] + [0, 1, 2, 3, 4]


def test_prune_vs_sorted(orc):
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(1, 3000))
        imp = rng.lognormal(0, 2, n).astype(np.float32)
        if trial % 2:  # heavy ties
            imp = np.round(imp, 1).astype(np.float32)
        imp[rng.integers(0, n, n // 10)] = 0.0
        k = np.sort(rng.integers(0, n + 1, 5)).astype(np.int64)
        kept = orc.prune_select(imp, k)
        order = sorted(range(n), key=lambda i: (-float(imp[i]), i))
        off = 0
        prev = set()
        for kt in k:
            want = sorted(order[:kt])
            got = kept[off:off + kt].tolist()
            off += kt
            assert got == want
            assert prev <= set(got)
            prev = set(got)


# ---------------------------------------------------------------- VQ
def test_vq_brute_force(orc):
    rng = np.random.default_rng(1)
    for n, D, K in [(500, 36, 64), (300, 1, 7), (200, 5, 1), (400, 36, 300)]:
        x = rng.laplace(0, 0.03, (n, D)).astype(np.float32)
        cb = x[rng.choice(n, K, replace=False)] if K <= n else rng.normal(0, 1, (K, D)).astype(np.float32)
        idx, dist = orc.vq_assign(x, cb)
        d = ((x[:, None, :].astype(np.float64) - cb[None, :, :].astype(np.float64)) ** 2).sum(-1)
        assert np.array_equal(idx, d.argmin(1).astype(np.int32))
        np.testing.assert_allclose(dist, d.min(1), rtol=1e-12)


def test_vq_self_and_duplicates(orc):
    rng = np.random.default_rng(2)
    cb = rng.normal(0, 1, (50, 36)).astype(np.float32)
    cb[30] = cb[10]  # duplicated codeword: the lower index wins
    idx, dist = orc.vq_assign(cb, cb)
    want = np.arange(50)
    want[30] = 10
    assert np.array_equal(idx, want) and (dist == 0).all()


# ---------------------------------------------------------------- ILP
def test_ilp_hand_case(orc):
    err = np.array([[4.0, 1.0], [3.0, 2.0]])
    size = np.array([[10, 20], [10, 20]])
    for solve in (orc.ilp_exhaustive, orc.ilp_dp):
        choice, obj, used = solve(err, size, 30)
        assert choice.tolist() == [1, 0] and obj == 4.0 and used == 30


def test_ilp_budget_edges(orc):
    rng = np.random.default_rng(4)
    err = np.sort(rng.uniform(0, 10, (5, 4)), axis=1)[:, ::-1].copy()
    size = np.sort(rng.integers(1, 50, (5, 4)), axis=1)
    for solve in (orc.ilp_exhaustive, orc.ilp_dp):
        big = solve(err, size, int(size.max(1).sum()) + 5)
        assert big[0].tolist() == list(np.argmin(err, axis=1))
        tight = solve(err, size, int(size.min(1).sum()))
        assert (size[np.arange(5), tight[0]] == size.min(1)).all()
        assert solve(err, size, int(size.min(1).sum()) - 1) is None


def test_ilp_exhaustive_vs_dp(orc):
    rng = np.random.default_rng(5)
    for trial in range(40):
        ncls = int(rng.integers(1, 6))
        nopt = int(rng.integers(1, 6))
        err = rng.uniform(0, 100, (ncls, nopt))
        size = rng.integers(0, 40, (ncls, nopt))
        if trial % 3 == 0:
            err[:, -1] = err[:, 0]  # exact ties across options
            size[:, -1] = size[:, 0]
        budget = int(rng.integers(0, 40 * ncls))
        a = orc.ilp_exhaustive(err, size, budget)
        b = orc.ilp_dp(err, size, budget)
        assert (a is None) == (b is None)
        if a is not None:
            assert a[1] == pytest.approx(b[1], rel=1e-12) and a[2] == b[2]
            assert a[0].tolist() == b[0].tolist()


def test_ilp_dp_vs_highs(orc):
    """The DP optimum equals scipy's MILP (HiGHS) optimum on medium tables."""
    from scipy.optimize import LinearConstraint, milp
    rng = np.random.default_rng(6)
    for trial in range(6):
        ncls, nopt = 30, 8
        err = np.sort(rng.lognormal(0, 2, (ncls, nopt)), axis=1)[:, ::-1].copy()
        size = np.sort(rng.integers(5, 400, (ncls, nopt)), axis=1)
        budget = int(rng.uniform(size.min(1).sum(), size.max(1).sum()))
        choice, obj, used = orc.ilp_dp(err, size, budget)
        A_eq = np.kron(np.eye(ncls), np.ones(nopt))
        cons = [LinearConstraint(A_eq, 1, 1), LinearConstraint(size.reshape(1, -1), 0, budget)]
        res = milp(err.ravel(), constraints=cons, integrality=np.ones(ncls * nopt),
                   bounds=(0, 1), options={"mip_rel_gap": 0})
        assert res.status == 0
        assert obj == pytest.approx(res.fun, rel=1e-9)
        assert used <= budget


def test_search_space_reading():
    """The paper's 2.96e722 options for (C, B, Q) = (10, 60, 16) is Q^(C*B):
    Q options per block, not (C*B)^Q."""
    assert 600 * math.log10(16) == pytest.approx(722 + math.log10(2.96), abs=2e-3)
    assert 16 * math.log10(600) < 50


def test_choose_ratio_rule(orc):
    rows = [
        {"tau": Fraction(1, 10), "size8": 40, "budget": 100, "obj": 1.0},   # skipped: 2*40 < 100
        {"tau": Fraction(2, 10), "size8": 60, "budget": 100, "obj": 5.0},
        {"tau": Fraction(3, 10), "size8": 80, "budget": 100, "obj": None},  # infeasible
        {"tau": Fraction(4, 10), "size8": 90, "budget": 100, "obj": 5.0},   # tie -> larger tau
        {"tau": Fraction(5, 10), "size8": 99, "budget": 100, "obj": 7.0},
    ]
    assert orc.choose_ratio(rows) == 3


# --------------------------------------------------------------- hierarchical solver
# Two channels x two groups of n = 10 elements, candidate bit-widths {2, 4};
# sizes are the linear n * b + 72 (92 and 112 bits).  Channel-level options:
# channel 0 at b = 2 costs loss 18 / 184 bits, at b = 4 loss 3 / 224 bits;
# channel 1 at b = 2 loss 7 / 184 bits, at b = 4 loss 5.5 / 224 bits.
HIER_ERR = np.array([[10.0, 1.0], [8.0, 2.0], [3.0, 2.5], [4.0, 3.0]])
HIER_SIZE = np.array([[92, 112]] * 4, dtype=np.int64)


def test_hierarchical_budget_split_by_hand(orc):
    # S_T = 400: only (2, 2) fits at the channel level (368 bits), so both
    # channels get 400 * 2 / 4 = 200 bits and keep b = 2 in every group
    choice, obj, used, qc, shares = orc.ilp_hierarchical(HIER_ERR, HIER_SIZE, 2, [2, 4], 400)
    assert choice.tolist() == [0, 0, 0, 0] and obj == 25.0 and used == 368
    assert qc.tolist() == [2, 2] and shares.tolist() == [200, 200]
    # the flat ILP spends the spare 32 bits on the best single upgrade (loss 16)
    flat = orc.ilp_exhaustive(HIER_ERR, HIER_SIZE, 400)
    assert flat[0].tolist() == [1, 0, 0, 0] and flat[1] == 16.0
    # S_T = 500: (4, 4) fits (448 bits), shares 250 each, every group at b = 4,
    # which is also the flat optimum
    choice, obj, used, qc, shares = orc.ilp_hierarchical(HIER_ERR, HIER_SIZE, 2, [2, 4], 500)
    assert choice.tolist() == [1, 1, 1, 1] and obj == 8.5 and used == 448 and shares.tolist() == [250, 250]
    assert orc.ilp_exhaustive(HIER_ERR, HIER_SIZE, 500)[1] == 8.5
    # S_T = 420: the channel level picks (4, 2) (loss 10, 408 bits); channel 1's
    # share 420 * 2 / 6 = 140 bits cannot hold its cheapest 184 bits
    assert orc.ilp_hierarchical(HIER_ERR, HIER_SIZE, 2, [2, 4], 420) is None


def test_hierarchical_never_beats_flat(orc):
    """Brute force on tiny random instances: the two-step result fits the
    budget, each channel's part is optimal for its share, and its loss is never
    below the flat optimum."""
    rng = np.random.default_rng(5)
    for _ in range(60):
        C, ng, nopt = int(rng.integers(1, 4)), int(rng.integers(1, 3)), int(rng.integers(1, 4))
        bl = sorted(rng.choice(np.arange(1, 17), nopt, replace=False).tolist())
        err = rng.random((C * ng, nopt)) * 10
        size = rng.integers(1, 30, (C * ng, nopt))
        budget = int(rng.integers(0, 40 * C * ng))
        r = orc.ilp_hierarchical(err, size, C, bl, budget, solve=orc.ilp_exhaustive)
        flat = orc.ilp_exhaustive(err, size, budget)
        if r is None:
            continue
        choice, obj, used, qc, shares = r
        assert used <= budget and flat is not None and obj >= flat[1] - 1e-12
        assert shares.sum() <= budget
        for c in range(C):
            sl = slice(c * ng, (c + 1) * ng)
            part = orc.ilp_exhaustive(err[sl], size[sl], int(shares[c]))
            assert part is not None and part[0].tolist() == choice[sl].tolist()


# ------------------------------------------------------------ calibrated search
def calib_tables(bits_b4, bits_b8, err_b4=5.0, err_b8=1.0):
    """One ratio, one channel, two groups of G = 10 elements, b in {4, 8}:
    linear sizes 112 / 152 bits, measured ceil(bits) + 72."""
    err = np.array([[[[err_b4, err_b8]] * 2]], dtype=np.float64)     # [T=1][C=1][2][2]
    bits = np.array([[[[bits_b4, bits_b8]] * 2]], dtype=np.float64)
    return err, bits


def test_calibrated_search_converges_by_hand(orc):
    # all-8 start measures 2 * 122 = 244 bits against the estimate 304, so
    # S_delta = -60 and the first ILP may use 310 linear bits: every group at
    # b = 8 (304), measured 244, within 5 % of S_T = 250
    err, bits = calib_tables(30.0, 50.0)
    r = orc.search_calibrated(err, bits, [20], 10, [4, 8], 250)
    assert r["status"].tolist() == [orc.SOLVED] and r["iters"].tolist() == [1]
    assert r["obj"][0] == 2.0 and r["actual"].tolist() == [244]
    assert r["best_t"] == 0 and r["best_bits"].tolist() == [[8, 8]]
    # doubling the all-8 size (488) stays below S_T = 1000: the ratio is skipped
    r = orc.search_calibrated(err, bits, [20], 10, [4, 8], 1000)
    assert r["status"].tolist() == [orc.SKIPPED] and r["iters"].tolist() == [0] and r["best_t"] == -1


def test_calibrated_search_oscillates_by_hand(orc):
    # measured sizes 80 (b = 4) and 150 (b = 8) per group, S_T = 240: all-8
    # measures 300 (estimate 304) -> S_delta = -4 -> limit 244 -> all b = 4
    # (224 linear bits), measured 160 -> S_delta = -64 -> limit 304 -> all
    # b = 8, measured 300 -> ... neither is within 5 %
    err, bits = calib_tables(8.0, 78.0)
    r = orc.search_calibrated(err, bits, [20], 10, [4, 8], 240, max_iter=5)
    assert r["status"].tolist() == [orc.UNCONVERGED] and r["iters"].tolist() == [5]
    assert r["obj"][0] == 10.0 and r["actual"].tolist() == [160] and r["best_t"] == -1
    r = orc.search_calibrated(err, bits, [20], 10, [4, 8], 240, max_iter=4)
    assert r["obj"][0] == 2.0 and r["actual"].tolist() == [300]


def test_calibrated_search_ratio_choice(orc):
    """Two converged ratios: the smaller loss wins; equal losses go to the larger k."""
    err, bits = calib_tables(30.0, 50.0)
    e2 = np.concatenate([err, err * 0.5], axis=0)
    b2 = np.concatenate([bits, bits], axis=0)
    r = orc.search_calibrated(e2, b2, [20, 20], 10, [4, 8], 250)
    assert r["best_t"] == 1 and r["obj"].tolist() == [2.0, 1.0]
    r = orc.search_calibrated(np.concatenate([err, err], axis=0), b2, [20, 20], 10, [4, 8], 250)
    assert r["best_t"] == 1  # tie, equal k: the later ratio


# ---------------------------------------------------------------- mini-batch k-means
def test_kmeans_step_by_hand(orc):
    """Centers 0 and 10 with one absorbed sample each, batch 1, 2, 9: 1 and 2
    go to center 0 (learning rates 1/2 then 1/3: 0 -> 0.5 -> 1.0), 9 to
    center 1 (rate 1/2: 10 -> 9.5)."""
    x = np.array([[1.0], [2.0], [9.0]], np.float32)
    cb = np.array([[0.0], [10.0]], np.float32)
    c, v, a = orc.kmeans_step(x, cb, [1, 1], [0, 1, 2])
    assert a.tolist() == [0, 0, 1] and v.tolist() == [3, 2]
    assert c[:, 0].tolist() == [1.0, 9.5]
    # a center that has absorbed nothing takes its first row, then the mean
    c, v, a = orc.kmeans_step(x, cb, [0, 5], [1, 0, 1])
    assert a.tolist() == [0, 0, 0] and v.tolist() == [3, 5]
    assert c[0, 0] == np.float32(5.0 / 3.0) and c[1, 0] == 10.0


def test_kmeans_step_is_the_running_mean(orc):
    """The per-sample updates of a batch equal the closed form
    (v c + sum of the center's rows) / (v + n) of the running mean."""
    rng = np.random.default_rng(8)
    x = rng.normal(0, 1, (300, 5)).astype(np.float32)
    cb = x[rng.choice(300, 7, replace=False)].copy()
    counts = rng.integers(0, 20, 7)
    batch = rng.integers(0, 300, 120)
    c, v, a = orc.kmeans_step(x, cb, counts, batch)
    for j in range(7):
        rows = x[batch[a == j]].astype(np.float64)
        assert v[j] == counts[j] + rows.shape[0]
        if rows.shape[0]:
            want = (counts[j] * cb[j].astype(np.float64) + rows.sum(0)) / v[j]
            np.testing.assert_allclose(c[j], want.astype(np.float32), rtol=3e-7, atol=1e-7)
        else:
            assert np.array_equal(c[j], cb[j])
    # the assignment is the exact nearest center of each batch row
    d = ((x[batch][:, None, :].astype(np.float64) - cb[None].astype(np.float64)) ** 2).sum(-1)
    assert np.array_equal(a, d.argmin(1))


def test_kmeans_step_batched(orc):
    """The batched running mean: the hand-worked step above gives the same
    centers (0 -> (1*0 + 1 + 2)/3 = 1, 10 -> (10 + 9)/2 = 9.5, and 5/3 for a
    center with nothing absorbed); on random data it agrees with the
    per-sample updates within FP32 rounding, assignments and counts equal."""
    x = np.array([[1.0], [2.0], [9.0]], np.float32)
    cb = np.array([[0.0], [10.0]], np.float32)
    c, v, a = orc.kmeans_step_batched(x, cb, [1, 1], [0, 1, 2])
    assert a.tolist() == [0, 0, 1] and v.tolist() == [3, 2]
    assert c[:, 0].tolist() == [1.0, 9.5]
    c, v, a = orc.kmeans_step_batched(x, cb, [0, 5], [1, 0, 1])
    assert c[0, 0] == np.float32(5.0 / 3.0) and c[1, 0] == 10.0 and v.tolist() == [3, 5]
    rng = np.random.default_rng(9)
    x = rng.normal(0, 1, (400, 6)).astype(np.float32)
    cb = x[rng.choice(400, 9, replace=False)].copy()
    counts = rng.integers(0, 30, 9)
    batch = rng.integers(0, 400, 200)
    cs, vs, as_ = orc.kmeans_step(x, cb, counts, batch)
    cbt, vb, ab = orc.kmeans_step_batched(x, cb, counts, batch)
    assert np.array_equal(as_, ab) and np.array_equal(vs, vb)
    np.testing.assert_allclose(cbt, cs, rtol=3e-7, atol=1e-7)
    # the rows of a center are summed one after another in batch order
    j = int(ab[0])
    mine = x[batch[ab == j]].astype(np.float64)
    seq = np.zeros(6)
    for r in mine:
        seq = seq + r
    want = ((np.float64(counts[j]) * cb[j].astype(np.float64) + seq) / np.float64(counts[j] + mine.shape[0]))
    assert np.array_equal(cbt[j], want.astype(np.float32))


def test_vq_retain_by_hand(orc):
    """130 remaining bits hold two 2-dim FP32 vectors (64 bits each): the two
    most important Gaussians (importance 5 at index 4, 4 at index 2) keep
    their own rows, appended in index order after the K = 3 codewords."""
    x = np.arange(10, dtype=np.float32).reshape(5, 2)
    cb = np.full((3, 2), -1.0, np.float32)
    idx = np.array([0, 1, 2, 0, 1], np.int32)
    ext, new, r = orc.vq_retain(x, [3, 1, 4, 1, 5], cb, idx, 130)
    assert r == 2 and new.tolist() == [0, 1, 3, 0, 4]
    assert ext.tolist() == cb.tolist() + [[4.0, 5.0], [8.0, 9.0]]
    # equal importance: the lower indices are kept; no budget keeps nothing
    ext, new, r = orc.vq_retain(x, [1, 1, 1, 1, 1], cb, idx, 128)
    assert r == 2 and new.tolist() == [3, 4, 2, 0, 1]
    assert orc.vq_retain(x, [1] * 5, cb, idx, 63)[2] == 0


# ----------------------------------------------------------------------- RAHT
def test_raht_paper_example(orc):
    """The paper's 2-D example: a1 = 1 at (0, 0) and a2 = 3 at (1, 0) merge along
    x (weights 1, 1): d1 = 4/sqrt 2, c1 = 2/sqrt 2 = sqrt 2; then d1 (weight 2)
    and a0 = 5 at (0, 1) along y: d2 = (sqrt 2 d1 + 5)/sqrt 3 = 3 sqrt 3,
    c2 = (sqrt 2 * 5 - d1)/sqrt 3 = sqrt 6.  One DC and two ACs."""
    coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]])
    assert orc.morton(coords, 1).tolist() == [0, 1, 2]
    out = orc.raht_forward(coords, np.array([[1.0, 3.0, 5.0]], np.float32), 1)
    np.testing.assert_allclose(out[0], [3 * math.sqrt(3), math.sqrt(2), math.sqrt(6)], rtol=1e-7)
    # one leaf: its value is the DC
    assert orc.raht_forward(np.array([[5, 2, 7]]), np.array([[2.5]], np.float32), 3).tolist() == [[2.5]]


def test_raht_invariants(orc):
    """Orthonormal: the energy is preserved and the DC is sqrt(N) times the mean;
    a constant attribute has (numerically) zero AC coefficients."""
    from paper_2604_26799_amd import synth
    coords = synth.voxels(700, 5, seed=3)
    coords = coords[np.argsort(orc.morton(coords, 5))]
    rng = np.random.default_rng(3)
    a = rng.normal(0, 1, (2, 700)).astype(np.float32)
    out = orc.raht_forward(coords, a, 5).astype(np.float64)
    a64 = a.astype(np.float64)
    np.testing.assert_allclose((out ** 2).sum(1), (a64 ** 2).sum(1), rtol=1e-5)
    np.testing.assert_allclose(out[:, 0], math.sqrt(700) * a64.mean(1), rtol=1e-5)
    const = orc.raht_forward(coords, np.full((1, 700), 2.0, np.float32), 5)
    assert np.abs(const[0, 1:]).max() < 1e-5 and const[0, 0] == pytest.approx(2.0 * math.sqrt(700), rel=1e-6)


def test_raht_depth2_by_hand(orc):
    """A 3-D example two levels deep, worked by hand from T_1.  Six voxels of a
    4 x 4 x 4 grid: p1 (0,0,0), p2 (1,0,0), p3 (0,1,0), p4 (1,0,1), p5 (3,2,0),
    p6 (2,3,1).  Morton codes (x in bit 3l, y in bit 3l+1, z in bit 3l+2):
    0, 1, 2, 5, 25, 30 -- the per-axis interleave (bit l + 2a) would give 0, 1,
    4, 17, 11, 30 and z in bit 3l gives 0, 4, 2, 5, 52, 51: other orders.  Level 0, x: p1 + p2 (weights 1, 1); y: that
    node (2) + p3 (1); z: that node (3) + p4 (1), and p5 + p6 (1, 1), which
    meet only at this axis.  Level 1, x: nothing; y: the two nodes (4, 2).
    Any other axis or level order changes the weights or the pairs, hence
    these numbers."""
    r2, r3, r6 = math.sqrt(2.0), math.sqrt(3.0), math.sqrt(6.0)
    coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 0, 1], [3, 2, 0], [2, 3, 1]])
    assert orc.morton(coords, 2).tolist() == [0, 1, 2, 5, 25, 30]
    a = [1.0, 3.0, -2.0, 5.0, 0.5, 4.0]
    l12 = (a[0] + a[1]) / r2
    h1 = (a[1] - a[0]) / r2
    l123 = (r2 * l12 + a[2]) / r3
    h2 = (r2 * a[2] - l12) / r3
    l1234 = (r3 * l123 + a[3]) / 2.0
    h3 = (r3 * a[3] - l123) / 2.0
    l56 = (a[4] + a[5]) / r2
    h4 = (a[5] - a[4]) / r2
    dc = (2.0 * l1234 + r2 * l56) / r6
    h5 = (2.0 * l56 - r2 * l1234) / r6
    want = [dc, h1, h2, h3, h4, h5]
    # closed forms of the same numbers: the DC is sqrt(6) times the mean, and
    # the first coefficients reduce to simple sums
    assert dc == pytest.approx(sum(a) / r6, rel=1e-15)
    assert h1 == pytest.approx(2.0 / r2, rel=1e-15)
    assert h2 == pytest.approx((2.0 * -2.0 - 4.0) / r6, rel=1e-15)
    assert h3 == pytest.approx((3.0 * 5.0 - 2.0) / (2.0 * r3), rel=1e-15)
    attr = np.array([a, [2.0] * 6], np.float32)
    out = orc.raht_forward(coords, attr, 2)
    np.testing.assert_allclose(out[0], np.array(want, np.float32), rtol=2e-7, atol=1e-7)
    # a constant channel: DC = 2 sqrt(6), every AC zero
    np.testing.assert_allclose(out[1], [2.0 * r6, 0, 0, 0, 0, 0], atol=1e-6)
