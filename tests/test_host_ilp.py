"""The library's host 0-1 ILP and reserve-ratio loop against the oracle (CPU)."""
import numpy as np
import pytest

from paper_2604_26799_amd import mgs, synth


def rand_table(rng, ncls, nopt, kind):
    if kind == "mono":  # loss falls and size grows with the option, like bit-widths
        err = np.sort(rng.lognormal(0, 2, (ncls, nopt)), axis=1)[:, ::-1].copy()
        size = np.sort(rng.integers(5, 400, (ncls, nopt)), axis=1)
    elif kind == "ties":
        err = rng.integers(0, 5, (ncls, nopt)).astype(np.float64)
        size = rng.integers(0, 6, (ncls, nopt)) * 10
    else:
        err = rng.uniform(0, 100, (ncls, nopt))
        size = rng.integers(0, 60, (ncls, nopt))
    return err, size


def test_hand_case():
    err = np.array([[4.0, 1.0], [3.0, 2.0]])
    size = np.array([[10, 20], [10, 20]])
    choice, obj, used = mgs.ilp_solve(err, size, 30)
    assert choice.tolist() == [1, 0] and obj == 4.0 and used == 30
    assert mgs.ilp_solve(err, size, 19) is None


@pytest.mark.parametrize("kind", ["mono", "ties", "free"])
def test_vs_exhaustive(orc, kind):
    rng = np.random.default_rng({"mono": 1, "ties": 2, "free": 3}[kind])
    for trial in range(150):
        ncls = int(rng.integers(1, 7))
        nopt = int(rng.integers(1, 6))
        err, size = rand_table(rng, ncls, nopt, kind)
        budget = int(rng.integers(0, max(1, size.sum(1).max() * ncls // 2 + 1)))
        a = orc.ilp_exhaustive(err, size, budget)
        b = mgs.ilp_solve(err, size, budget)
        assert (a is None) == (b is None), (trial, budget)
        if a is not None:
            assert b[1] == a[1] and b[2] == a[2], (trial, a, b)
            assert b[0].tolist() == a[0].tolist(), (trial, a, b)


def test_vs_dp_medium(orc):
    rng = np.random.default_rng(9)
    for trial in range(25):
        ncls = int(rng.integers(10, 60))
        nopt = int(rng.integers(2, 16))
        err, size = rand_table(rng, ncls, nopt, "mono" if trial % 2 else "free")
        lo, hi = int(size.min(1).sum()), int(size.max(1).sum())
        budget = int(rng.uniform(lo, hi))
        a = orc.ilp_dp(err, size, budget)
        b = mgs.ilp_solve(err, size, budget)
        assert (a is None) == (b is None)
        if a is not None:
            assert b[1] == pytest.approx(a[1], rel=1e-12) and b[2] == a[2]
            if b[0].tolist() != a[0].tolist():  # only possible on an exact tie
                assert b[1] == a[1]


def _rounding_broken_class(rng):
    """Three options whose middle one stays on the lower hull (by the hull
    test's products) while the two efficiencies, as quotients, rise along it:
    near-collinear points where rounding decides.  Such a class makes the LP
    step fall back from the sorted selection to the heap merge."""
    while True:
        sb = int(rng.integers(1, 51))
        sc = sb + int(rng.integers(1, 51))
        ea = 1.0 + float(rng.random())
        slope = float(rng.random())
        eb = ea - slope * sb * (1 + float(rng.choice([1e-16, -1e-16, 2e-16, -2e-16])))
        ec = ea - slope * sc
        if not ea > eb > ec or (eb - ea) * float(sc) >= (ec - ea) * float(sb):
            continue
        if (eb - ec) / float(sc - sb) > (ea - eb) / float(sb):
            return [ea, eb, ec], [0, sb, sc]


def test_rounding_broken_hull(orc):
    rng = np.random.default_rng(17)
    for trial in range(40):
        ncls = int(rng.integers(2, 7)) if trial < 30 else int(rng.integers(20, 50))
        err, size = rand_table(rng, ncls, 3, "mono")
        for c in rng.choice(ncls, size=max(1, ncls // 2), replace=False):
            err[c], size[c] = _rounding_broken_class(rng)
        lo, hi = int(size.min(1).sum()), int(size.max(1).sum())
        budget = int(rng.integers(lo, hi + 1))
        a = orc.ilp_exhaustive(err, size, budget) if ncls <= 6 else orc.ilp_dp(err, size, budget)
        b = mgs.ilp_solve(err, size, budget)
        assert (a is None) == (b is None), trial
        if a is not None:
            assert b[1] == pytest.approx(a[1], rel=1e-12) and b[2] == a[2], (trial, a, b)
            if b[0].tolist() != a[0].tolist():  # only possible on an exact tie
                assert b[1] == a[1]


def test_large_vs_highs():
    """Thousands of classes (the size of a real sweep's table) against HiGHS."""
    from scipy.optimize import LinearConstraint, milp
    rng = np.random.default_rng(12)
    ncls, nopt = 1500, 16
    err, size = rand_table(rng, ncls, nopt, "mono")
    budget = int(0.35 * size.min(1).sum() + 0.65 * size.max(1).sum())
    choice, obj, used = mgs.ilp_solve(err, size, budget)
    assert used <= budget
    A_eq = np.kron(np.eye(ncls), np.ones(nopt))
    res = milp(err.ravel(), constraints=[LinearConstraint(A_eq, 1, 1),
                                         LinearConstraint(size.reshape(1, -1), 0, budget)],
               integrality=np.ones(ncls * nopt), bounds=(0, 1),
               options={"mip_rel_gap": 0, "time_limit": 120})
    assert res.status == 0
    assert obj <= res.fun * (1 + 1e-9)
    assert obj == pytest.approx(res.fun, rel=1e-9)


def test_budget_edges():
    rng = np.random.default_rng(4)
    err, size = rand_table(rng, 40, 8, "mono")
    big = mgs.ilp_solve(err, size, int(size.max(1).sum()) + 5)
    assert big[0].tolist() == list(np.argmin(err, axis=1))
    tight = mgs.ilp_solve(err, size, int(size.min(1).sum()))
    assert (size[np.arange(40), tight[0]] == size.min(1)).all()
    assert mgs.ilp_solve(err, size, int(size.min(1).sum()) - 1) is None
    with pytest.raises(mgs.MgsError):
        bad = err.copy()
        bad[3, 2] = np.nan
        mgs.ilp_solve(bad, size, 1000)


def test_size_table_modes(orc):
    rng = np.random.default_rng(1)
    bits = rng.uniform(0, 5000, (30, 5))
    bits[3] = 0.0
    bits[4, 1] = 17.0  # exact integer stays as is
    n = rng.integers(1, 4096, 30)
    bl = [2, 4, 5, 8, 16]
    assert np.array_equal(mgs.size_table(bits, mode=0), orc.size_table(bits))
    assert np.array_equal(mgs.size_table(bits, n, bl, mode=1), orc.size_table(bits, n, bl, "linear"))


def test_search_vs_oracle(orc):
    """Reserve-ratio loop + ILP on the oracle's tables of a small scene."""
    w = synth.SweepWorkload("t", 6000, 11, synth.ratios_uniform(synth.Fraction(2, 10), synth.Fraction(9, 10), 5),
                            512, [2, 4, 6, 8])
    attr, imp = w.make()
    k = w.k
    kept = orc.prune_select(imp, k)
    tab = orc.quant_sweep(attr, imp, kept, k, w.group, w.bits)
    raw_bits = w.n * w.channels * 32
    for ratio in (8, 12, 20, 40):
        budget = raw_bits // ratio
        res = mgs.search(w.n, w.channels, k, w.group, w.bits, tab["err"], tab["bits"], budget, solve_all=True)
        fast = mgs.search(w.n, w.channels, k, w.group, w.bits, tab["err"], tab["bits"], budget)
        assert fast["best_t"] == res["best_t"]
        if res["best_t"] >= 0:
            assert np.array_equal(fast["best_bits"], res["best_bits"])
            # ratios left unsolved had a lower bound above the chosen optimum
            for t in np.where(fast["status"] == mgs.SEARCH_PRUNED)[0]:
                assert res["obj"][t] > res["obj"][res["best_t"]]
        rows = []
        for t in range(len(k)):
            ng = (int(k[t]) + w.group - 1) // w.group
            e = tab["err"][t, :, :ng].reshape(-1, len(w.bits))
            s = orc.size_table(tab["bits"][t, :, :ng].reshape(-1, len(w.bits)))
            size8 = int(s[:, w.bits.index(8)].sum())
            sol = orc.ilp_dp(e, s, budget) if 2 * size8 >= budget else None
            rows.append({"tau": int(k[t]), "size8": size8, "budget": budget,
                         "obj": None if sol is None else sol[1], "sol": sol})
            if 2 * size8 < budget:
                assert np.isnan(res["obj"][t])
            elif sol is None:
                assert np.isnan(res["obj"][t])
            else:
                assert res["obj"][t] == pytest.approx(sol[1], rel=1e-12)
                assert res["used"][t] == sol[2]
        best = orc.choose_ratio(rows)
        if best is None:
            assert res["best_t"] == -1
            continue
        assert res["best_t"] == best
        want = np.asarray(w.bits, np.uint8)[rows[best]["sol"][0]].reshape(w.channels, -1)
        assert np.array_equal(res["best_bits"], want)


def test_search_rejects_invalid_tables():
    """A loss that is not finite, or an entropy size that is negative or not
    finite, fails the whole search, whether its ratio is solved, pruned or
    skipped (its doubled all-8-bit size below the budget)."""
    rng = np.random.default_rng(23)
    N, C, G, bits = 4000, 3, 256, [2, 4, 8]
    k = [400, 2000, 4000]
    T, gm = len(k), (max(k) + G - 1) // G
    err = np.sort(rng.uniform(0, 10, (T, C, gm, 3)), axis=3)[..., ::-1].copy()
    bt = np.zeros((T, C, gm, 3))
    for t, kt in enumerate(k):
        for g in range((kt + G - 1) // G):
            n = min(G, kt - g * G)
            bt[t, :, g] = np.array(bits) * n * rng.uniform(0.3, 0.9, (C, 1))
    ngs = [(kt + G - 1) // G for kt in k]
    s8 = [int(np.ceil(bt[t, :, :ngs[t], 2]).sum()) + 72 * C * ngs[t] for t in range(T)]
    smin2 = int(np.ceil(bt[2, :, :ngs[2], 0]).sum()) + 72 * C * ngs[2]
    budget = (smin2 + s8[1]) // 2  # ratio 0 skipped (2 * s8 < budget), the others feasible
    assert 2 * s8[0] < budget <= 2 * s8[1] and smin2 <= budget
    ok = mgs.search(N, C, k, G, bits, err, bt, budget)
    assert ok["status"][0] == mgs.SEARCH_SKIPPED and ok["best_t"] >= 1
    # the smallest admissible ratio (solved ahead of the others) made to lose:
    # it is reported pruned, as any ratio whose bound exceeds the optimum
    e = err.copy()
    e[1] *= 100.0
    fast = mgs.search(N, C, k, G, bits, e, bt, budget)
    full = mgs.search(N, C, k, G, bits, e, bt, budget, solve_all=True)
    assert fast["best_t"] == full["best_t"] == 2
    assert fast["status"].tolist() == [mgs.SEARCH_SKIPPED, mgs.SEARCH_PRUNED, mgs.SEARCH_SOLVED]
    assert np.isnan(fast["obj"][1]) and fast["used"][1] == 0
    assert full["obj"][1] > full["obj"][2] and fast["obj"][2] == full["obj"][2]
    for t in range(T):
        for what in ("err_nan", "err_inf", "bits_neg", "bits_nan", "bits8_nan"):
            e, b = err.copy(), bt.copy()
            g = ngs[t] - 1
            if what == "err_nan":
                e[t, 1, g, 0] = np.nan
            elif what == "err_inf":
                e[t, 2, 0, 1] = np.inf
            elif what == "bits_neg":
                b[t, 0, g, 1] = -1.0
            elif what == "bits_nan":
                b[t, 2, g, 0] = np.nan
            else:
                b[t, 1, 0, 2] = np.nan
            with pytest.raises(mgs.MgsError) as ex:
                mgs.search(N, C, k, G, bits, e, b, budget)
            assert ex.value.code == mgs.EINVAL, (t, what)
        # linear sizes ignore the entropy table
        b = bt.copy()
        b[t, 0, 0, 0] = np.nan
        mgs.search(N, C, k, G, bits, err, b, budget, size_mode=1)


@pytest.mark.parametrize("kind", ["mono", "ties", "free"])
def test_hierarchical_vs_oracle(orc, kind):
    """The library's two-step solver against the oracle's (channel level under
    the whole budget, shares floor(S_T Q_c / sum Q_c), per-channel ILPs)."""
    rng = np.random.default_rng({"mono": 11, "ties": 12, "free": 13}[kind])
    for _ in range(40):
        C, ng, nopt = int(rng.integers(1, 6)), int(rng.integers(1, 6)), int(rng.integers(1, 6))
        bl = sorted(rng.choice(np.arange(1, 17), nopt, replace=False).tolist())
        err, size = rand_table(rng, C * ng, nopt, kind)
        budget = int(rng.integers(0, int(size.max(axis=1).sum()) + 2))
        want = orc.ilp_hierarchical(err, size, C, bl, budget)
        got = mgs.ilp_hierarchical(err, size, C, bl, budget)
        if want is None:
            assert got is None
            continue
        assert got is not None
        assert got[0].tolist() == want[0].tolist()
        assert got[1] == pytest.approx(want[1], rel=1e-12, abs=1e-12)
        assert got[2] == want[2]
        assert got[3].tolist() == want[3].tolist() and got[4].tolist() == want[4].tolist()
        flat = mgs.ilp_solve(err, size, budget)
        assert flat is not None and got[1] >= flat[1] - 1e-9 and got[2] <= budget


def test_calibrated_search_vs_oracle(orc):
    """Algorithm 1 with the linear estimator and measured entropy sizes, on the
    oracle's tables of a small scene, for budgets that converge, oscillate and
    skip ratios; with 8 among the candidates and without."""
    for bits in ([2, 4, 6, 8], [3, 5, 7]):
        w = synth.SweepWorkload("t", 5000, 11, synth.ratios_uniform(synth.Fraction(2, 10), synth.Fraction(9, 10), 4),
                                512, bits)
        attr, imp = w.make()
        attr = np.ascontiguousarray(attr[:5])  # five channels keep the oracle's DP small
        w.channels = 5
        k = w.k
        kept = orc.prune_select(imp, k)
        tab = orc.quant_sweep(attr, imp, kept, k, w.group, w.bits)
        raw_bits = w.n * w.channels * 32
        for ratio in (6, 9, 14, 25, 60):
            budget = raw_bits // ratio
            for tol in (50000, 5000):
                want = orc.search_calibrated(tab["err"], tab["bits"], k, w.group, w.bits, budget, tol_ppm=tol,
                                             max_iter=6)
                got = mgs.search_calibrated(w.n, w.channels, k, w.group, w.bits, tab["err"], tab["bits"], budget,
                                            tol_ppm=tol, max_iter=6)
                assert got["status"].tolist() == want["status"].tolist(), (bits, ratio, tol)
                assert got["iters"].tolist() == want["iters"].tolist()
                assert got["actual"].tolist() == want["actual"].tolist()
                np.testing.assert_allclose(got["obj"], want["obj"], rtol=1e-12, equal_nan=True)
                assert got["best_t"] == want["best_t"]
                if want["best_t"] >= 0:
                    assert np.array_equal(got["best_bits"], want["best_bits"])
