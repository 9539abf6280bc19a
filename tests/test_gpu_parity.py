"""HIP path vs the CPU oracle, element by element, through the C ABI.

Bar: codes, histograms, kept indices and VQ indices bit-exact; loss tables
within 4e-6 relative, size tables as below.  On the fast path the kernels form each loss
term in FP32 (on values scaled by an exact power of two), sum up to EPT
<= 32 of them per thread and then the 64 lanes of a wavefront in FP32
before the FP64 sum over waves, so a group's loss carries a relative error
of at most (32 + 9) * 2^-24 ~ 2.4e-6 (wavefront sums that overflow or could
have lost terms to underflow are recomputed in FP64); the tests assert
ERR_REL = 4e-6.  Literal-division and underflowed-step groups keep
FP64 terms.  The size is the FP64 entropy; for bit-widths with more bins
than a sixteenth of the group it comes from entropy increments on a 2^-K grid (exact
sums), which adds an absolute error of at most G * 2^-(K+1) bits (K from
increment_bits below); the tests assert 1e-9 relative plus that bound.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2604_26799_amd import mgs, synth

pytestmark = pytest.mark.gpu
ERR_REL = 4e-6
BITS_REL = 1e-9


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    mgs.lib()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def hist_fits(attr, k, G, bits, limit=2e7):
    """Debug histograms only when T*C*Gmax*sum(2^b) bins stay small."""
    slots = len(k) * attr.shape[0] * max(1, (int(np.max(k)) + G - 1) // G)
    return slots * sum(2 ** b for b in bits) <= limit


def gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=True):
    out = mgs.quant_sweep(dev(torch, attr), dev(torch, imp), dev(torch, kept.astype(np.int32)), k, G, bits,
                          want_hist=hist)
    torch.cuda.synchronize()
    return {key: (host(v) if v is not None else None) for key, v in out.items()}


def increment_bits(G):
    """Grid exponent of the entropy increments (kept in step with the library)."""
    top = G * math.log2(max(G, 2)) + G + 1.0
    return 52 - math.ceil(math.log2(top))


def assert_tables(got, want, hist=True, G=None):
    assert got["err"].shape == want["err"].shape
    atol_bits = 1e-9 if G is None else max(1e-9, G * 2.0 ** -(increment_bits(G) + 1))
    nan = np.isnan(want["err"])
    assert np.array_equal(np.isnan(got["err"]), nan)
    assert np.array_equal(np.isnan(got["bits"]), np.isnan(want["bits"]))
    np.testing.assert_allclose(got["err"][~nan], want["err"][~nan], rtol=ERR_REL, atol=1e-300)
    np.testing.assert_allclose(got["bits"][~nan], want["bits"][~nan], rtol=BITS_REL, atol=atol_bits)
    gn = ~np.isnan(want["gmin"])
    assert np.array_equal(got["gmin"][gn], want["gmin"][gn])
    assert np.array_equal(got["gmax"][gn], want["gmax"][gn])
    if hist:
        assert np.array_equal(got["hist"].view(np.uint32), want["hist"])


# ------------------------------------------------------------------ sweep
def test_sweep_small_workload(torch, orc):
    """N=50,000, 11 channels, 4 ratios, G=4096, b in 4..8: every table entry and bin."""
    w = synth.workload("small")
    attr, imp = w.make()
    k = w.k
    kept = orc.prune_select(imp, k)
    want = orc.quant_sweep(attr, imp, kept, k, w.group, w.bits, want_hist=True)
    got = gpu_sweep(torch, attr, imp, kept, k, w.group, w.bits)
    assert_tables(got, want, G=w.group)


@pytest.mark.parametrize("n,C,G,bits", [
    (2000, 2, 1, [1, 2, 9]),                  # one-element groups (constant)
    (400, 2, 37, list(range(1, 17))),         # ragged tiny groups, every b (b >= 15 packed)
    (3000, 2, 300, [3, 9, 15, 16]),
    (20000, 20, 300, [3, 9, 15, 16]),         # (tables only)
    (20000, 20, 1000, [2, 5]),
    (20000, 8, 4097, [1, 4, 8, 12, 16]),      # just over a power of two
    (20000, 11, 9000, [2, 16]),
    (40000, 8, 16384, list(range(1, 17))),
    (70000, 4, 65535, [1, 8, 16]),            # the largest group
])
def test_sweep_shapes(torch, orc, n, C, G, bits):
    attr, imp = synth.scene(n, 20, seed=G)
    attr = np.ascontiguousarray(attr[:C])
    k = np.clip(np.array([0, 1, n - 1, n, 7777, G], np.int64), 0, n)
    kept = orc.prune_select(imp, k)
    hist = hist_fits(attr, k, G, bits)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits, want_hist=hist)
    got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=hist)
    assert_tables(got, want, hist=hist, G=G)


def adversarial_scene(n, seed):
    """Constant groups, lattice values, huge and tiny magnitudes, subnormals,
    ranges whose scale underflows, and offsets that make |Z| > 2^23."""
    rng = np.random.default_rng(seed)
    C = 8
    a = np.empty((C, n), np.float32)
    a[0] = 2.5                                                     # constant channel
    a[1] = (rng.integers(0, 64, n) * 0.125).astype(np.float32)     # lattice
    a[2] = rng.normal(0, 1, n) * 1e30                              # huge
    a[3] = rng.normal(0, 1, n) * 1e-30                             # tiny (S subnormal at high b)
    a[4] = (rng.integers(0, 3, n) * np.float32(1e-45)).astype(np.float32)  # subnormal steps
    a[5] = 1.0e4 + rng.normal(0, 1e-3, n)                          # large offset: |Z| > 2^23
    a[6] = np.where(rng.random(n) < 0.5, -0.0, 0.0)                # signed zeros
    a[7] = rng.laplace(0, 0.05, n)
    imp = rng.lognormal(0, 2, n).astype(np.float32)
    imp[rng.random(n) < 0.05] = 0.0
    return a, imp


@pytest.mark.parametrize("G", [64, 1000, 4096])
def test_sweep_adversarial(torch, orc, G):
    attr, imp = adversarial_scene(12000, G)
    k = np.array([12000, 5000, 3], np.int64)
    bits = [1, 2, 7, 11, 15, 16]
    kept = orc.prune_select(imp, k)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits, want_hist=False)
    got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=False)
    assert_tables(got, want, hist=False, G=G)
    # histograms of the adversarial channels at the small bit-widths
    hb = [1, 2, 7, 11]
    want = orc.quant_sweep(attr, imp, kept, k, G, hb, want_hist=True)
    got = gpu_sweep(torch, attr, imp, kept, k, G, hb, hist=True)
    assert_tables(got, want, hist=True, G=G)


def quotient_tie_scene(G, bits, C, seed):
    """Channels whose values put x / S_b + Z_b on a rounding tie (a half
    integer) or a few ulps away from one, for every listed b, plus the group's
    min and max; the rest of the group uniform in [min, max]."""
    rng = np.random.default_rng(seed)
    f32 = np.float32
    attr = np.empty((C, G), f32)
    for c in range(C):
        mn, mx = f32(-rng.uniform(0.01, 50.0)), f32(rng.uniform(0.01, 50.0))
        if c % 3 == 2:  # far from zero with a narrow range
            mn, mx = f32(1000.0 + rng.uniform(0, 1)), f32(1003.0 + rng.uniform(0, 1))
        R = f32(mx - mn)
        vals = [mn, mx]
        for b in bits:
            P = f32(2.0 ** b)
            S = f32(R / P)
            Z = f32(np.rint(P - f32(mx / S)))
            for j in rng.integers(0, 2 ** b, size=90):
                x = f32(f32(f32(j + 0.5) - Z) * S)  # x / S close to the tie j + 0.5 - Z
                for step in range(-3, 4):
                    y = x
                    for _ in range(abs(step)):
                        y = np.nextafter(y, f32(np.inf) if step > 0 else f32(-np.inf))
                    if mn <= y <= mx:
                        vals.append(y)
        vals = np.array(vals[:G], f32)
        fill = rng.uniform(float(mn), float(mx), size=G - len(vals)).astype(f32)
        row = np.concatenate([vals, np.clip(fill, mn, mx)])
        rng.shuffle(row)
        attr[c] = row
    imp = rng.uniform(0.1, 2.0, size=G).astype(f32)
    return attr, imp


def literal_codes(x, b):
    """The FP32 quantizer of one group, literally (numpy FP32 operations are
    correctly rounded); `nudge` moves x / R one ulp up before the scaling."""
    f32 = np.float32
    mn, mx = x.min(), x.max()
    R, P = f32(mx - mn), f32(2.0 ** b)
    S = f32(R / P)
    Z = f32(np.rint(P - f32(mx / S)))
    u = (x / R).astype(f32)
    out = []
    for uu in (u, np.nextafter(u, f32(np.inf))):
        t = (uu * P).astype(f32) + Z  # uu * P is exact: P is a power of two
        out.append(np.rint(np.clip(t, f32(0), P - 1)))
    return out


def test_sweep_quotient_ties(torch, orc):
    """Codes on and next to rounding ties for every bit-width: the kernel's
    x / R (one reciprocal per group, two FMA corrections per element) must be
    the correctly rounded quotient, else codes here move.  The scene is
    checked to be sensitive: moving x / R by one ulp changes codes."""
    G, C = 4096, 6
    bits = [1, 3, 8, 12, 16]
    attr, imp = quotient_tie_scene(G, bits, C, seed=77)
    moved = sum(int(np.sum(a != b)) for c in range(C) for bb in bits for a, b in [literal_codes(attr[c], bb)])
    assert moved > 100, moved
    k = np.array([G], np.int64)
    kept = np.arange(G, dtype=np.int32)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits, want_hist=True)
    got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=True)
    assert_tables(got, want, hist=True, G=G)


def test_sweep_every_shape_identical(torch, orc):
    """Launch shapes (threads, elements per thread, LDS capacity, channels per
    tile, chunked, persistent grid) change nothing beyond the summation order
    of the loss:
    every shape matches the oracle, shapes agree with each other within the
    loss bound (sizes to 1e-12), group bounds exactly, and a repeated launch
    of one shape is bit-identical."""
    attr, imp = synth.scene(30000, 20, seed=9)
    k = np.array([30000, 17777, 4097], np.int64)
    G, bits = 4096, [2, 5, 9, 13, 16]
    kept = orc.prune_select(imp, k)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits)
    first = None
    shapes = [(256, 16, 0, 0), (512, 8, 0, 1), (1024, 4, 65536, 3), (512, 16, 98304, 7),
              (1024, 8, 0, 20), (256, 32, 65536, 2), (512, 16, 65536, 1),
              # persistent grids: tiles from the per-XCD counters
              (512, 16, 98304, 4, 1), (1024, 8, 0, 0, 1), (256, 32, 65536, 2, 1), (1024, 16, 0, 1, 1)]
    try:
        for sh in shapes:
            mgs.sweep_set_shape(G, len(bits), max(bits), *sh)
            got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=False)
            assert_tables(got, want, hist=False, G=G)
            again = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=False)
            for key in ("err", "bits", "gmin", "gmax"):
                assert np.array_equal(got[key], again[key], equal_nan=True), (sh, key)
            if first is None:
                first = got
            else:
                for key in ("gmin", "gmax"):
                    assert np.array_equal(got[key], first[key], equal_nan=True), (sh, key)
                ok = ~np.isnan(first["err"])
                np.testing.assert_allclose(got["err"][ok], first["err"][ok], rtol=2 * ERR_REL)
                np.testing.assert_allclose(got["bits"][ok], first["bits"][ok], rtol=1e-12, atol=1e-9)
        # a group larger than the shape's capacity takes the chunked kernel
        want = orc.quant_sweep(attr, imp, kept, k, 16384, bits)
        for persist in (0, 1):
            mgs.sweep_set_shape(16384, len(bits), max(bits), 512, 16, 0, 5, persist)
            got = gpu_sweep(torch, attr, imp, kept, k, 16384, bits, hist=False)
            assert_tables(got, want, hist=False, G=16384)
    finally:
        mgs.sweep_set_shape(G, len(bits), max(bits), 0, 0, 0, 0)
        mgs.sweep_set_shape(16384, len(bits), max(bits), 0, 0, 0, 0)


def test_sweep_split_tail(torch, orc):
    """A persistent launch of one scene with whole-group tiles ends each XCD's
    range of groups in tiles of a few channels.  323 groups of 256 (the last
    one ragged) over 11 channels: every range holds whole and split groups,
    and the last range has fewer groups than the others.  The tables match
    the oracle and, bit for bit, the same sweep in one-channel tiles."""
    G, bits = 256, [2, 5, 9]
    k = np.array([323 * G - 100], np.int64)
    attr, imp = synth.scene(int(k[0]) + 7000, 11, seed=12)
    kept = orc.prune_select(imp, k)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits)
    try:
        mgs.sweep_set_shape(G, len(bits), max(bits), 256, 1, 0, 0, 1)
        got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=False)
        assert_tables(got, want, hist=False, G=G)
        mgs.sweep_set_shape(G, len(bits), max(bits), 256, 1, 0, 1, 0)
        plain = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=False)
        for key in ("err", "bits", "gmin", "gmax"):
            assert np.array_equal(got[key], plain[key], equal_nan=True), key
    finally:
        mgs.sweep_set_shape(G, len(bits), max(bits), 0, 0, 0, 0)


@pytest.mark.parametrize("scale", [1e-38, 1e38])
def test_sweep_extreme_weights(torch, orc, scale):
    """Importance weights at the ends of the FP32 range: the FP32 loss terms
    underflow to subnormals or their sums overflow, and the kernel's FP64
    recomputation of those wavefront sums keeps every table on the FP64
    definition."""
    attr, imp = synth.scene(30000, 20, seed=11)
    attr = np.ascontiguousarray(attr[:4])
    w = (imp / imp.max() * np.float32(scale)).astype(np.float32)
    assert np.isfinite(w).all()
    k = np.array([30000, 9000], np.int64)
    G, bits = 4096, [2, 8, 13, 16]
    kept = orc.prune_select(w, k)
    want = orc.quant_sweep(attr, w, kept, k, G, bits, want_hist=False)
    got = gpu_sweep(torch, attr, w, kept, k, G, bits, hist=False)
    assert_tables(got, want, hist=False, G=G)


def crowded_scene(n, seed):
    """Channels with few distinct values: bins that collect far more than 256
    elements at every bit-width."""
    rng = np.random.default_rng(seed)
    a = np.empty((3, n), np.float32)
    a[0] = rng.integers(0, 5, n) * np.float32(0.5)                     # 5 values
    a[1] = np.where(rng.random(n) < 0.9, 0.0, rng.normal(0, 1, n))     # 90% in one bin
    a[2] = rng.integers(0, 300, n).astype(np.float32) ** 2 * 1e-4      # 300 values, uneven
    imp = rng.lognormal(0, 1, n).astype(np.float32)
    return a, imp


@pytest.mark.parametrize("G,shape", [(8192, None), (8192, (512, 16, 65536, 1)),
                                     (16384, None), (16384, (512, 16, 65536, 2))])
def test_sweep_crowded_bins(torch, orc, G, shape):
    """Incremental entropy with counts past the LDS increment table, on whole
    histograms and on bin windows (the small LDS capacity splits b >= 15)."""
    attr, imp = crowded_scene(40000, G)
    k = np.array([40000, 20000, G + 5], np.int64)
    bits = [2, 9, 13, 14, 15, 16]
    kept = orc.prune_select(imp, k)
    want = orc.quant_sweep(attr, imp, kept, k, G, bits, want_hist=True)
    try:
        if shape:
            mgs.sweep_set_shape(G, len(bits), max(bits), *shape)
        got = gpu_sweep(torch, attr, imp, kept, k, G, bits, hist=True)
    finally:
        if shape:
            mgs.sweep_set_shape(G, len(bits), max(bits), 0, 0, 0, 0)
    assert_tables(got, want, hist=True, G=G)


def test_sweep_nonfinite_flag(torch, orc):
    attr, imp = synth.scene(5000, 11, seed=1)
    attr[3, 100] = np.nan
    k = np.array([5000], np.int64)
    kept = np.arange(5000, dtype=np.int32)
    with pytest.raises(mgs.MgsError) as e:
        gpu_sweep(torch, attr, imp, kept, k, 1024, [4, 8], hist=False)
    assert e.value.code == mgs.ENONFINITE
    out = mgs.quant_sweep(dev(torch, attr), dev(torch, imp), dev(torch, kept), k, 1024, [4, 8], check=False)
    err = host(out["err"])
    assert np.isnan(err[0, 3, 0]).all() and np.isfinite(err[0, 3, 1:]).all() and np.isfinite(err[0, 2]).all()


def sampled_tiles(orc, attr, imp, kept, k, G, bits, got, picks):
    """Oracle one tile at a time: the tile's slice as its own one-group sweep."""
    offs = np.concatenate([[0], np.cumsum(k)])
    for t, c, g in picks:
        J = kept[offs[t]:offs[t + 1]][g * G:(g + 1) * G]
        sub = orc.quant_sweep(attr[c:c + 1, J], imp[J], np.arange(J.size, dtype=np.int32),
                              np.array([J.size]), G, bits)
        np.testing.assert_allclose(got["err"][t, c, g], sub["err"][0, 0, 0], rtol=ERR_REL)
        np.testing.assert_allclose(got["bits"][t, c, g], sub["bits"][0, 0, 0], rtol=BITS_REL,
                                   atol=max(1e-9, G * 2.0 ** -(increment_bits(G) + 1)))
        assert got["gmin"][t, c, g] == sub["gmin"][0, 0, 0]
        assert got["gmax"][t, c, g] == sub["gmax"][0, 0, 0]


def test_sweep_medium_workload_sampled(torch, orc):
    """N=1e6, 20 channels, 16 ratios, G=8192, b in 2..16 (full size) with the
    default launch shape (eager): sampled tiles plus NaN padding and whole-table
    invariants.  The autotuned, graph-replayed launch the benchmark times is
    compared with the oracle on every tile in test_gpu_search_parity.py."""
    w = synth.workload("medium")
    attr, imp = w.make()
    k = w.k
    kept_d = mgs.prune_select(dev(torch, imp), k)
    kept = host(kept_d)
    np.testing.assert_array_equal(kept, orc.prune_select(imp, k))
    got = gpu_sweep(torch, attr, imp, kept, k, w.group, w.bits, hist=False)
    rng = np.random.default_rng(0)
    picks = []
    for t in (0, 7, 15):
        ng = (int(k[t]) + w.group - 1) // w.group
        for g in (0, ng - 1, int(rng.integers(0, ng))):
            picks.append((t, int(rng.integers(0, w.channels)), g))
        assert np.isnan(got["err"][t, :, ng:]).all()
        assert np.isfinite(got["err"][t, :, :ng]).all()
    sampled_tiles(orc, attr, imp, kept, k, w.group, w.bits, got, picks)
    # loss nonincreasing in b over the whole table (1e-6 slack for FP32 rounding of t)
    e = got["err"]
    ok = ~np.isnan(e[..., 0])
    assert (e[ok][:, 1:] <= e[ok][:, :-1] * (1 + 1e-6)).all()
    n_per = np.minimum(w.group, k[:, None] - np.arange(e.shape[2])[None, :] * w.group)  # [T][Gmax]
    n_all = np.broadcast_to(n_per[:, None, :], e.shape[:3])[ok]
    assert (got["bits"][ok] <= np.asarray(w.bits)[None, :] * n_all[:, None] * (1 + 1e-12) + 1e-6).all()
    assert (got["bits"][ok] <= np.log2(n_all)[:, None] * n_all[:, None] * (1 + 1e-12) + 1e-6).all()


# ------------------------------------------------------------------ pruning
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prune_small(torch, orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 70000))
    imp = rng.lognormal(0, 2, n).astype(np.float32)
    if seed == 1:
        imp = np.round(imp).astype(np.float32)  # heavy ties
    if seed == 2:
        imp[rng.random(n) < 0.3] = 0.0
        imp[rng.random(n) < 0.1] = -0.0
        imp[rng.random(n) < 0.05] = -rng.lognormal(0, 1, n)[: 1].astype(np.float32)
    k = np.array(sorted(rng.integers(0, n + 1, 7).tolist()) + [n, 0, 1], np.int64)
    got = host(mgs.prune_select(dev(torch, imp), k))
    np.testing.assert_array_equal(got, orc.prune_select(imp, k))


def test_prune_large_workload(torch, orc):
    """N=5.3e6 with 32 ratios (328k tied importance values at this size)."""
    w = synth.workload("large")
    rng = np.random.default_rng(0)
    imp = rng.lognormal(0.0, 2.0, w.n).astype(np.float32)
    k = w.k
    got = host(mgs.prune_select(dev(torch, imp), k))
    np.testing.assert_array_equal(got, orc.prune_select(imp, k))


@pytest.mark.parametrize("ties", [False, True])
def test_prune_max_ratios(torch, orc, ties):
    """64 keep counts (the maximum) over 2x10^5 keys: the compaction blocks then
    take two ratios each; unsorted and repeated counts, 0 and n included."""
    rng = np.random.default_rng(21 + int(ties))
    n = 200_000
    imp = rng.lognormal(0, 2, n).astype(np.float32)
    if ties:
        imp = np.round(imp * 4).astype(np.float32)
    k = rng.integers(0, n + 1, 64).astype(np.int64)
    k[:4] = [0, n, 1, k[5]]
    got = host(mgs.prune_select(dev(torch, imp), k))
    np.testing.assert_array_equal(got, orc.prune_select(imp, k))


def test_prune_nonfinite(torch):
    imp = np.ones(1000, np.float32)
    imp[5] = np.inf
    with pytest.raises(mgs.MgsError) as e:
        mgs.prune_select(dev(torch, imp), [10])
    assert e.value.code == mgs.ENONFINITE


# ------------------------------------------------------------------ final codes
@pytest.mark.parametrize("G", [1, 100, 4096, 16384])
def test_quantize_dequantize(torch, orc, G):
    attr, imp = synth.scene(60000, 20, seed=3)
    adv, _ = adversarial_scene(60000, 4)
    attr = np.concatenate([attr, adv]).astype(np.float32)
    C = attr.shape[0]
    kept = orc.prune_select(imp, [45000])
    ng = (kept.size + G - 1) // G
    bw = np.random.default_rng(G).integers(1, 17, (C, ng)).astype(np.uint8)
    codes, mn, mx = orc.quantize(attr, kept, G, bw)
    gc, gmn, gmx = mgs.quantize(dev(torch, attr), dev(torch, kept), G, dev(torch, bw))
    np.testing.assert_array_equal(host(gc).view(np.uint16), codes)
    assert np.array_equal(host(gmn), mn) and np.array_equal(host(gmx), mx)
    xh = orc.dequantize(codes, G, bw, mn, mx)
    gx = host(mgs.dequantize(gc, G, dev(torch, bw), gmn, gmx))
    assert np.array_equal(gx, xh)  # numeric equality (+0 == -0)


def test_sweep_codes_match_quantize(torch, orc):
    """The sweep's histograms are the histograms of the final quantizer's codes."""
    attr, imp = synth.scene(9000, 11, seed=8)
    G, bits = 2048, [3, 9, 16]
    kept = np.arange(9000, dtype=np.int32)
    got = gpu_sweep(torch, attr, imp, kept, np.array([9000]), G, bits)
    ng = (9000 + G - 1) // G
    off = 0
    for i, b in enumerate(bits):
        bw = np.full((11, ng), b, np.uint8)
        gc, _, _ = mgs.quantize(dev(torch, attr), dev(torch, kept), G, dev(torch, bw))
        codes = host(gc).view(np.uint16)
        for c in range(11):
            for g in range(ng):
                h = np.bincount(codes[c, g * G:(g + 1) * G], minlength=2 ** b)
                assert np.array_equal(got["hist"][0, c, g, off:off + 2 ** b].view(np.uint32), h)
        off += 2 ** b


# ------------------------------------------------------------------ VQ
@pytest.mark.parametrize("n,D,K,seed", [
    (5000, 36, 4096, 0), (3000, 36, 100, 1), (2000, 1, 7, 2), (777, 5, 1, 3),
    (4000, 46, 333, 4), (1000, 64, 50, 5), (64, 36, 32, 6), (0, 36, 10, 7),
    (1500, 8, 77, 8), (1200, 12, 64, 9)])
def test_vq_small(torch, orc, n, D, K, seed):
    rng = np.random.default_rng(seed)
    x = rng.laplace(0, 0.03, (n, D)).astype(np.float32)
    cb = rng.laplace(0, 0.03, (K, D)).astype(np.float32)
    if n >= K:
        cb[: K // 2] = x[rng.choice(n, K // 2, replace=False)]
    idx, dist, nfb = mgs.vq_assign(dev(torch, x), dev(torch, cb))
    want_i, want_d = orc.vq_assign(x, cb)
    np.testing.assert_array_equal(host(idx), want_i)
    np.testing.assert_array_equal(host(dist), want_d)


@pytest.mark.parametrize("D", [36, 8])
def test_vq_unaligned_rows(torch, orc, D):
    """Rows that start 4 bytes past a 16-byte boundary take the per-element load
    path (the float4 path needs D % 4 == 0 and aligned rows); same results."""
    rng = np.random.default_rng(12)
    n, K = 2500, 300
    x = rng.laplace(0, 0.03, (n, D)).astype(np.float32)
    cb = rng.laplace(0, 0.03, (K, D)).astype(np.float32)
    buf = torch.zeros(n * D + 1, dtype=torch.float32, device="cuda")
    buf[1:].copy_(torch.from_numpy(x.reshape(-1)))
    xv = buf[1:].view(n, D)
    assert xv.data_ptr() % 16 == 4
    idx, dist, _ = mgs.vq_assign(xv, dev(torch, cb))
    want_i, want_d = orc.vq_assign(x, cb)
    np.testing.assert_array_equal(host(idx), want_i)
    np.testing.assert_array_equal(host(dist), want_d)


def test_vq_duplicates_and_self(torch, orc):
    rng = np.random.default_rng(11)
    cb = rng.laplace(0, 0.03, (500, 36)).astype(np.float32)
    cb[400:450] = cb[0:50]   # duplicated codewords: lowest index wins
    x = np.concatenate([cb, cb + np.float32(1e-7), rng.laplace(0, 0.03, (3000, 36)).astype(np.float32)])
    idx, dist, _ = mgs.vq_assign(dev(torch, x), dev(torch, cb))
    want_i, want_d = orc.vq_assign(x, cb)
    np.testing.assert_array_equal(host(idx), want_i)
    np.testing.assert_array_equal(host(dist), want_d)
    assert (host(idx)[400:450] == np.arange(50)).all()


@pytest.mark.parametrize("K,D", [(33, 36), (70, 36), (1, 8), (100, 5)])
def test_vq_zero_rows_against_padding(torch, orc, K, D):
    """Rows of zeros score ||sigma c_j||^2 >= 0 against every real codeword;
    the codebook is padded to whole 64-codeword chunks, and a padding codeword
    that scored 0 would set the running minimum below every real score and
    hide the winner.  Zero rows, rows of one codeword and random rows, with a
    row count that leaves the last workgroup partly empty."""
    rng = np.random.default_rng(41 + K)
    cb = (rng.laplace(0, 0.3, (K, D)) + np.float32(0.5)).astype(np.float32)
    x = rng.laplace(0, 0.3, (777, D)).astype(np.float32)
    x[::3] = 0.0
    x[1::5] = cb[rng.integers(0, K, x[1::5].shape[0])]
    idx, dist, _ = mgs.vq_assign(dev(torch, x), dev(torch, cb))
    want_i, want_d = orc.vq_assign(x, cb)
    np.testing.assert_array_equal(host(idx), want_i)
    np.testing.assert_array_equal(host(dist), want_d)


@pytest.mark.parametrize("case", ["x_far_larger", "x_far_smaller", "huge_codebook"])
def test_vq_operand_ranges(torch, orc, case):
    """The MFMA operands are sigma x and sigma c in FP16 with sigma set by the
    largest codeword norm: rows far larger than the codebook leave FP16 (exact
    scan), rows far smaller fall below its normal range (covered by the
    bound), and a huge codeword sets a tiny scale for the others."""
    rng = np.random.default_rng(31)
    cb = rng.laplace(0, 0.5, (700, 36)).astype(np.float32)
    x = rng.laplace(0, 0.5, (2000, 36)).astype(np.float32)
    if case == "x_far_larger":
        x[::7] *= np.float32(1e6)
    elif case == "x_far_smaller":
        x[::3] *= np.float32(1e-7)
    else:
        cb[5] = np.float32(1e30)
        x[:50] = cb[rng.integers(0, 700, 50)] + np.float32(1e-3)
    idx, dist, nfb = mgs.vq_assign(dev(torch, x), dev(torch, cb))
    want_i, want_d = orc.vq_assign(x, cb)
    np.testing.assert_array_equal(host(idx), want_i)
    np.testing.assert_array_equal(host(dist), want_d)
    if case == "x_far_larger":
        assert int(host(nfb)[0]) >= x[::7].shape[0]  # every scaled-out row took the exact scan


def test_vq_workload_sampled(torch, orc):
    """N=3e6 x 36 dims, K=4096 (the benchmarked launch); a 20k-row sample checked
    bit-exactly against the FP64 brute force, plus rows that equal codewords."""
    x, cb = synth.vq_data(3_000_000, 36, 4096, seed=0)
    idx, dist, nfb = mgs.vq_assign(dev(torch, x), dev(torch, cb))
    gi, gd = host(idx), host(dist)
    rng = np.random.default_rng(1)
    rows = rng.choice(x.shape[0], 20000, replace=False)
    want_i, want_d = orc.vq_assign(x[rows], cb)
    np.testing.assert_array_equal(gi[rows], want_i)
    np.testing.assert_array_equal(gd[rows], want_d)
    assert (gi >= 0).all() and (gi < 4096).all()
    assert int(host(nfb)[0]) < x.shape[0] // 1000  # exact full scans stay rare


def test_kmeans_steps(torch, orc):
    """Mini-batch k-means iterations on SH-like vectors: assignments, counts and
    centers bit-identical to the oracle's batched running mean (each center's
    rows summed in batch order), centers within FP32 rounding of the
    per-sample updates, and a repeat of the same step gives the same bits;
    every iteration starts both sides from the library's state."""
    x, cb = synth.vq_data(20_000, 36, 128, seed=4)
    rng = np.random.default_rng(4)
    counts = np.zeros(128, np.int64)
    counts[::3] = 7  # some centers have absorbed samples already
    xd = dev(torch, x)
    cbd = dev(torch, cb)
    cd = dev(torch, counts)
    for it in range(3):
        batch = rng.integers(0, x.shape[0], 4096)
        c0, v0 = host(cbd).copy(), host(cd).copy()
        # the same step twice from the same state: identical bits
        again_c, again_v = dev(torch, c0), dev(torch, v0)
        mgs.kmeans_step(xd, again_c, again_v, dev(torch, batch))
        a = mgs.kmeans_step(xd, cbd, cd, dev(torch, batch))
        torch.cuda.synchronize()
        assert np.array_equal(host(again_c), host(cbd)) and np.array_equal(host(again_v), host(cd)), it
        bc, bv, ba = orc.kmeans_step_batched(x, c0, v0, batch)
        assert np.array_equal(host(a), ba), it
        assert np.array_equal(host(cd), bv), it
        assert np.array_equal(host(cbd), bc), it
        wc, wv, wa = orc.kmeans_step(x, c0, v0, batch)
        assert np.array_equal(host(a), wa), it
        np.testing.assert_allclose(host(cbd), wc, rtol=2.5e-7, atol=1e-9)
    # an empty batch changes nothing
    c0 = host(cbd).copy()
    mgs.kmeans_step(xd, cbd, cd, dev(torch, np.zeros(0, np.int64)))
    assert np.array_equal(host(cbd), c0)
    # a row index outside [0, N) is reported
    with pytest.raises(mgs.MgsError) as e:
        mgs.kmeans_step(xd, cbd, cd, dev(torch, np.array([0, x.shape[0]], np.int64)))
    assert e.value.code == mgs.ENONFINITE


@pytest.mark.parametrize("remaining", [0, 32 * 36 * 7 + 5, 32 * 36 * 5000, 10 ** 12])
def test_vq_retain(torch, orc, remaining):
    """Budget-first retention after the assignment: extended codebook and index
    table equal the oracle's (copies, so bit for bit)."""
    x, cb = synth.vq_data(30_000, 36, 256, seed=6)
    imp = np.random.default_rng(6).lognormal(0, 2, x.shape[0]).astype(np.float32)
    imp[::97] = imp[0]  # ties
    idx0, _ = orc.vq_assign(x, cb)
    idx = dev(torch, idx0)
    ext, r = mgs.vq_retain(dev(torch, x), dev(torch, imp), dev(torch, cb), idx, remaining)
    torch.cuda.synchronize()
    wext, widx, wr = orc.vq_retain(x, imp, cb, idx0, remaining)
    assert r == wr
    assert np.array_equal(host(ext), wext)
    assert np.array_equal(host(idx), widx)


@pytest.mark.parametrize("n,depth,C", [(1, 4, 2), (3, 1, 1), (2000, 6, 3), (6000, 10, 2), (5000, 8, 40),
                                       (40000, 14, 20), (4096, 21, 1)])
def test_raht(torch, orc, n, depth, C):
    """RAHT forward: every coefficient bit-identical to the oracle (same FP64
    operations, FP32 storage); inverse: back to the attributes within FP32
    rounding, also from the oracle's coefficients."""
    from paper_2604_26799_amd import synth
    coords = synth.voxels(n, depth, seed=n) if n > 3 else np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]])[:n]
    codes = orc.morton(coords, depth)
    order = np.argsort(codes)
    coords, codes = coords[order], codes[order]
    a = np.random.default_rng(n).normal(0, 1, (C, n)).astype(np.float32)
    cd = dev(torch, codes.view(np.int64))
    got = mgs.raht(cd, dev(torch, a), depth)
    torch.cuda.synchronize()
    want = orc.raht_forward(coords, a, depth)
    assert np.array_equal(host(got), want)
    back = host(mgs.raht(cd, got, depth, inverse=True))
    np.testing.assert_allclose(back, a, rtol=1e-5, atol=1e-5)
    back2 = host(mgs.raht(cd, dev(torch, want), depth, inverse=True))
    np.testing.assert_allclose(back2, a, rtol=1e-5, atol=1e-5)


def test_raht_rejects_unsorted_codes(torch, orc):
    codes = np.array([3, 1, 2], np.int64)
    with pytest.raises(mgs.MgsError) as e:
        mgs.raht(dev(torch, codes), dev(torch, np.ones((1, 3), np.float32)), 2)
    assert e.value.code == mgs.ENONFINITE


@pytest.mark.parametrize("n,depth,C,G,bits", [(30000, 10, 3, 4096, [2, 5, 8, 12, 16]),
                                               (100000, 14, 20, 8192, list(range(2, 17)))])
def test_raht_then_sweep(torch, orc, n, depth, C, G, bits):
    """The sweep over RAHT AC coefficients (DC kept in floating point, unit
    weights) against the oracle's RAHT followed by the oracle's sweep: every
    table entry and the search's allocation on both tables."""
    from paper_2604_26799_amd import synth
    coords = synth.voxels(n, depth, seed=n)
    codes = orc.morton(coords, depth)
    order = np.argsort(codes)
    coords, codes = coords[order], codes[order]
    attr, _ = synth.scene(n, 20, seed=depth)
    attr = np.ascontiguousarray(attr[:C])
    coef, tab = mgs.raht_sweep(dev(torch, codes.view(np.int64)), dev(torch, attr), depth, G, bits)
    torch.cuda.synchronize()
    want_coef = orc.raht_forward(coords, attr, depth)
    assert np.array_equal(host(coef), want_coef)
    want = orc.quant_sweep(want_coef, np.ones(n, np.float32), np.arange(1, n, dtype=np.int32),
                           np.array([n - 1]), G, bits)
    got = {key: host(v) for key, v in tab.items() if v is not None}
    assert_tables(got, want, hist=False, G=G)
    budget = (n - 1) * C * 32 // 20
    a = mgs.search(n - 1, C, [n - 1], G, bits, got["err"], got["bits"], budget)
    b = mgs.search(n - 1, C, [n - 1], G, bits, want["err"], want["bits"], budget)
    assert a["best_t"] == b["best_t"] == 0
    assert np.array_equal(a["best_bits"], b["best_bits"])


def test_kmeans_one_center_takes_all(torch, orc):
    """Every batch row nearest to one center (a run of 20,000 rows summed in
    batch order) and centers that get nothing: bit-identical to the oracle's
    batched running mean."""
    rng = np.random.default_rng(14)
    x = rng.normal(0, 0.01, (30_000, 36)).astype(np.float32)
    cb = np.full((16, 36), 100.0, np.float32)
    cb[5] = 0.0
    counts = np.arange(16, dtype=np.int64)
    batch = rng.integers(0, x.shape[0], 20_000)
    cbd, cd = dev(torch, cb), dev(torch, counts)
    a = mgs.kmeans_step(dev(torch, x), cbd, cd, dev(torch, batch))
    torch.cuda.synchronize()
    bc, bv, ba = orc.kmeans_step_batched(x, cb, counts, batch)
    assert (ba == 5).all() and np.array_equal(host(a), ba)
    assert np.array_equal(host(cd), bv) and np.array_equal(host(cbd), bc)
