"""Batched sweep (several scenes in one launch) and graph-captured replay,
through the C ABI, against the per-scene sweep and the CPU oracle.

Bar: every table of a batched launch is bit-identical to the same scene's
own mgs_quant_sweep; graph replays are bit-identical to eager launches on the
same inputs, also after the inputs change between replays."""
import numpy as np
import pytest

from paper_2604_26799_amd import mgs, synth

pytestmark = pytest.mark.gpu

G, BITS = 4096, [2, 5, 9, 13, 16]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    mgs.lib()
    return _t


def scene(torch, orc, n, C, fracs, seed):
    attr, imp = synth.scene(n, 11 if C <= 11 else 20, seed=seed)
    attr = np.ascontiguousarray(attr[:C])
    k = np.array([max(1, int(n * f)) for f in fracs], np.int64)
    kept = orc.prune_select(imp, k)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return {"attr": dev(attr), "imp": dev(imp), "kept": dev(kept.astype(np.int32)), "k": k,
            "host": (attr, imp, kept)}


def same(a, b):
    return all(np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy(), equal_nan=True)
               for key in ("err", "bits", "gmin", "gmax"))


def test_multi_scene_equals_single_and_oracle(torch, orc):
    scenes = [scene(torch, orc, 30000, 11, [0.3, 0.5, 0.9], 1),
              scene(torch, orc, 12000, 20, [0.2, 1.0], 2),
              scene(torch, orc, 5000, 3, [0.05, 0.6, 0.7, 0.95], 3),
              scene(torch, orc, 40, 7, [0.5], 4)]              # one tiny ragged group
    outs = mgs.quant_sweep_multi(scenes, G, BITS)
    torch.cuda.synchronize()
    for sc, out in zip(scenes, outs):
        alone = mgs.quant_sweep(sc["attr"], sc["imp"], sc["kept"], sc["k"], G, BITS)
        torch.cuda.synchronize()
        assert same(out, alone)
        attr, imp, kept = sc["host"]
        want = orc.quant_sweep(attr, imp, kept, sc["k"], G, BITS)
        nan = np.isnan(want["err"])
        err = out["err"].cpu().numpy()
        assert np.array_equal(np.isnan(err), nan)
        np.testing.assert_allclose(err[~nan], want["err"][~nan], rtol=4e-6)
        np.testing.assert_allclose(out["bits"].cpu().numpy()[~nan], want["bits"][~nan], rtol=1e-9, atol=1e-6)


def test_multi_scene_split_tail(torch, orc):
    """A persistent launch with all channels per tile takes the scenes'
    groups in sequence and ends each XCD's range of them in tiles of a few
    channels (355 groups of 256: whole and split groups in every range,
    ranges across scene boundaries, a shorter last range).  Every scene's
    tables equal those of the same launch in one-channel tiles, bit for bit,
    and the oracle's."""
    g, bits = 256, [2, 5, 9]
    scenes = [scene(torch, orc, 40000, 6, [0.3, 0.9], 21), scene(torch, orc, 25000, 6, [0.5, 1.0], 22),
              scene(torch, orc, 7000, 6, [0.7], 23)]
    try:
        mgs.sweep_set_shape(g, len(bits), max(bits), 256, 1, 0, 0, 1)
        outs = mgs.quant_sweep_multi(scenes, g, bits)
        torch.cuda.synchronize()
        mgs.sweep_set_shape(g, len(bits), max(bits), 256, 1, 0, 1, 0)
        plain = mgs.quant_sweep_multi(scenes, g, bits)
        torch.cuda.synchronize()
    finally:
        mgs.sweep_set_shape(g, len(bits), max(bits), 0, 0, 0, 0)
    for sc, out, pl in zip(scenes, outs, plain):
        assert same(out, pl)
        attr, imp, kept = sc["host"]
        want = orc.quant_sweep(attr, imp, kept, sc["k"], g, bits)
        nan = np.isnan(want["err"])
        err = out["err"].cpu().numpy()
        assert np.array_equal(np.isnan(err), nan)
        np.testing.assert_allclose(err[~nan], want["err"][~nan], rtol=4e-6)
        np.testing.assert_allclose(out["bits"].cpu().numpy()[~nan], want["bits"][~nan], rtol=1e-9, atol=1e-6)
        assert np.array_equal(out["gmin"].cpu().numpy()[~np.isnan(want["gmin"])],
                              want["gmin"][~np.isnan(want["gmin"])])


def test_multi_scene_histograms(torch, orc):
    scenes = [scene(torch, orc, 9000, 4, [0.5, 1.0], 5), scene(torch, orc, 6000, 2, [0.3], 6)]
    bits = [1, 3, 7]
    outs = mgs.quant_sweep_multi(scenes, 1000, bits, want_hist=True)
    torch.cuda.synchronize()
    for sc, out in zip(scenes, outs):
        attr, imp, kept = sc["host"]
        want = orc.quant_sweep(attr, imp, kept, sc["k"], 1000, bits, want_hist=True)
        assert np.array_equal(out["hist"].cpu().numpy().view(np.uint32), want["hist"])


def test_graph_replay_matches_eager(torch, orc):
    """Capture once, replay three times with the inputs changed (and the
    outputs cleared) in between; each replay equals an eager launch."""
    s = torch.cuda.Stream()
    a = scene(torch, orc, 20000, 6, [0.4, 0.8], 7)
    b = scene(torch, orc, 7000, 5, [0.5, 1.0], 8)
    single_ws = mgs.workspace(1 << 22, a["attr"].device)
    jobs, outs = mgs.sweep_jobs([a, b], G, BITS)
    multi_ws = mgs.workspace(mgs.lib().mgs_quant_sweep_multi_ws_bytes(jobs, len(jobs)), a["attr"].device)
    gm = mgs.gmax_groups(a["k"], G)
    one = mgs.sweep_tables(len(a["k"]), 6, gm, len(BITS), a["attr"].device)
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        g1 = mgs.capture(lambda: mgs.quant_sweep(a["attr"], a["imp"], a["kept"], a["k"], G, BITS, ws=single_ws,
                                                 out=one, stream=s, check=False), s)
        g2 = mgs.capture(lambda: mgs.quant_sweep_multi(None, G, BITS, ws=multi_ws, stream=s, check=False,
                                                       jobs=jobs), s)
        for r in range(3):
            for sc in (a, b):
                sc["attr"].mul_(1.25).add_(0.5 * r)
            for t in [one, *outs]:
                for key in ("err", "bits", "gmin", "gmax"):
                    t[key].fill_(-7.0)
            g1.launch(s)
            g2.launch(s)
            s.synchronize()
            eager_a = mgs.quant_sweep(a["attr"], a["imp"], a["kept"], a["k"], G, BITS, stream=s)
            eager_b = mgs.quant_sweep(b["attr"], b["imp"], b["kept"], b["k"], G, BITS, stream=s)
            s.synchronize()
            assert same(one, eager_a), r
            assert same(outs[0], eager_a), r
            assert same(outs[1], eager_b), r
    g1.close()
    g2.close()
