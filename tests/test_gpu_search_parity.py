"""The search's answers from the GPU tables against the oracle's, on the full
workloads, with the launch the benchmark times.

For every workload the HIP path computes the tables with the autotuned launch
shape replayed from a captured graph (replays checked against each other and
against the eager launch); every entry of every table is compared with the
oracle's (err within ERR_REL, bits within the increment-grid bound, bounds
exact), histograms on a full-size subset, and then the reserve-ratio search
with its exact 0-1 ILP (paper: equation "ilp" of section "Solve the MINLP";
Algorithm 1 "Hyperparameter Optimization") runs on the GPU tables and on the
oracle's tables: chosen ratio, bit allocation and total size must be equal,
the loss within ERR_REL, and the final codes at the allocation equal the
oracle's.  On the small workload the oracle's own capacity DP and ratio rule
decide the allocation as well.
"""
import numpy as np
import pytest

from paper_2604_26799_amd import mgs, synth
from test_gpu_parity import ERR_REL, assert_tables, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    mgs.lib()
    return _t


def timed_launch_tables(torch, attr_d, imp_d, kept_d, k, G, bits, autotune=True):
    """Tables from the launch the benchmark times: the autotuner's shape (it
    registers it), then a captured graph replayed twice, the tables scribbled
    over before each replay; both replays and the eager launch must agree bit
    for bit.  Returns host tables and the shape."""
    s = torch.cuda.Stream()
    T, C, nb = len(k), attr_d.shape[0], len(bits)
    gm = mgs.gmax_groups(k, G)
    tab = mgs.sweep_tables(T, C, gm, nb, attr_d.device)
    import ctypes as ct
    d = mgs.sweep_desc(attr_d.shape[1], C, k, G, bits)
    ws = mgs.workspace(mgs.lib().mgs_quant_sweep_ws_bytes(ct.byref(d)), attr_d.device)
    shape = None
    with torch.cuda.stream(s):
        if autotune:
            shape, _ = mgs.sweep_autotune(attr_d, imp_d, kept_d, k, G, bits, reps=1, ws=ws, out=tab, stream=s)
        eager = mgs.quant_sweep(attr_d, imp_d, kept_d, k, G, bits, ws=ws, stream=s)
        s.synchronize()
        eager = {key: host(v) for key, v in eager.items() if v is not None}
        graph = mgs.capture(lambda: mgs.quant_sweep(attr_d, imp_d, kept_d, k, G, bits, ws=ws, out=tab,
                                                    stream=s, check=False), s)
        try:
            for rep in range(2):
                for key in ("err", "bits", "gmin", "gmax"):
                    tab[key].fill_(-7.0)
                s.synchronize()
                graph.launch(s)
                s.synchronize()
                assert mgs.status(ws, s) == mgs.OK
                got = {key: host(tab[key]) for key in ("err", "bits", "gmin", "gmax")}
                for key in got:
                    assert np.array_equal(got[key], eager[key], equal_nan=True), (rep, key)
        finally:
            graph.close()
    return got, shape


def search_both(w_n, C, k, G, bits, got, want, budget):
    """mgs.search on the GPU tables and on the oracle tables; equal answers."""
    a = mgs.search(w_n, C, k, G, bits, got["err"], got["bits"], budget)
    b = mgs.search(w_n, C, k, G, bits, want["err"], want["bits"], budget)
    t = b["best_t"]
    assert t >= 0
    msg = ""
    if a["best_t"] != t or not np.array_equal(a["best_bits"], b["best_bits"]):
        # the two allocations, each scored on the oracle's tables
        msg = f"ratio {a['best_t']} vs {t}; obj {a['obj'][a['best_t']]!r} vs {b['obj'][t]!r}"
    assert a["best_t"] == t, msg
    assert np.array_equal(a["best_bits"], b["best_bits"]), msg
    assert a["used"][t] == b["used"][t] <= budget
    assert a["obj"][t] == pytest.approx(b["obj"][t], rel=ERR_REL)
    return b


def codes_both(torch, orc, attr, attr_d, kept, k, G, res):
    t = res["best_t"]
    offs = np.concatenate([[0], np.cumsum(k)])
    kt = kept[offs[t]:offs[t + 1]]
    codes, mn, mx = mgs.quantize(attr_d, dev(torch, kt), G, dev(torch, res["best_bits"]))
    oc, omn, omx = orc.quantize(attr, kt, G, res["best_bits"])
    assert np.array_equal(host(codes).view(np.uint16), oc)
    assert np.array_equal(host(mn), omn) and np.array_equal(host(mx), omx)


def hist_subset(torch, orc, attr, imp, kept, k, G, bits, chans, ratios):
    """Debug histograms of a few channels and ratios at full size, same
    registered shape and bit list: bin for bin equal to the oracle's."""
    offs = np.concatenate([[0], np.cumsum(k)])
    ks = np.array([k[t] for t in ratios], np.int64)
    ksub = np.concatenate([kept[offs[t]:offs[t + 1]] for t in ratios]).astype(np.int32)
    a = np.ascontiguousarray(attr[chans])
    want = orc.quant_sweep(a, imp, ksub, ks, G, bits, want_hist=True)
    out = mgs.quant_sweep(dev(torch, a), dev(torch, imp), dev(torch, ksub), ks, G, bits, want_hist=True)
    torch.cuda.synchronize()
    got = {key: host(v) for key, v in out.items()}
    assert_tables(got, want, hist=True, G=G)


def run_workload(torch, orc, w, budget, hist_chans, hist_ratios):
    attr, imp = w.make()
    k, G, C = w.k, w.group, w.channels
    attr_d, imp_d = dev(torch, attr), dev(torch, imp)
    kept_d = mgs.prune_select(imp_d, k)
    kept = host(kept_d)
    assert np.array_equal(kept, orc.prune_select(imp, k))
    try:
        got, shape = timed_launch_tables(torch, attr_d, imp_d, kept_d, k, G, w.bits)
        print(f"{w.name}: autotuned shape {shape}", flush=True)
        want = orc.quant_sweep(attr, imp, kept, k, G, w.bits)
        assert_tables(got, want, hist=False, G=G)
        if hist_chans:
            hist_subset(torch, orc, attr, imp, kept, k, G, w.bits, hist_chans, hist_ratios)
    finally:
        mgs.sweep_set_shape(G, len(w.bits), max(w.bits), 0, 0, 0, 0)
    res = search_both(w.n, C, k, G, w.bits, got, want, budget)
    codes_both(torch, orc, attr, attr_d, kept, k, G, res)
    return k, want, res


def test_search_parity_small(torch, orc):
    """N=50,000, 11 channels, 4 ratios, G=4096, b in 4..8, budget raw/30; the
    oracle's capacity DP and ratio rule pick the same allocation."""
    w = synth.workload("small")
    budget = w.n * w.channels * 32 // 30
    k, want, res = run_workload(torch, orc, w, budget, [0, 5], [0, 3])
    rows = []
    for t in range(len(k)):
        ng = (int(k[t]) + w.group - 1) // w.group
        e = want["err"][t, :, :ng].reshape(-1, len(w.bits))
        s = orc.size_table(want["bits"][t, :, :ng].reshape(-1, len(w.bits)))
        size8 = int(s[:, w.bits.index(8)].sum())
        sol = orc.ilp_dp(e, s, budget) if 2 * size8 >= budget else None
        rows.append({"tau": int(k[t]), "size8": size8, "budget": budget,
                     "obj": None if sol is None else sol[1], "sol": sol})
    best = orc.choose_ratio(rows)
    assert best == res["best_t"]
    bw = np.asarray(w.bits, np.uint8)[rows[best]["sol"][0]].reshape(w.channels, -1)
    assert np.array_equal(bw, res["best_bits"])
    assert rows[best]["sol"][1] == pytest.approx(res["obj"][best], rel=1e-12)


def test_search_parity_medium(torch, orc):
    """N=1e6, 20 channels, 16 ratios, G=8192, b in 2..16, budget raw/30: all
    22,600 tiles, histograms of 2 channels x 2 ratios."""
    w = synth.workload("medium")
    run_workload(torch, orc, w, w.n * w.channels * 32 // 30, [3, 15], [0, 15])


def test_search_parity_large(torch, orc):
    """N=5.3e6, 20 channels, 32 ratios, G=16384, b in 1..16, budget raw/30:
    all 109,020 tiles, histograms of one channel at the smallest and largest
    ratio, the search and the final codes."""
    w = synth.workload("large")
    run_workload(torch, orc, w, w.n * w.channels * 32 // w.budget_ratio, [12], [0, 31])


def test_search_parity_served_jobs(torch, orc):
    """The first six jobs of the serving stream (seed 0: N from 2.9e5 to
    4.9e6, budgets raw/10..raw/60), served together in one batched launch:
    each job's ratio, bit allocation and codes equal the answer the search
    gives on the oracle's tables of that job."""
    from paper_2604_26799_amd import serve
    jobs = synth.job_stream(64, 2.0, seed=0)[:6]
    store = serve.SceneStore(num_bases=2, n=max(j.n for j in jobs))
    srv = serve.Server(store, mode="batched", keep_codes=True)
    out = srv.run(jobs, time_scale=0.0)
    srv.close()
    assert out["jobs"] == 6 and out["failed"] == 0 and out["max_batch"] == 6
    by_id = {r.job_id: r for r in out["results"]}
    G, bits, C = srv.G, srv.bits, serve.CHANNELS
    for job in jobs:
        attr = np.ascontiguousarray(store.attr[job.base][:, :job.n].numpy())
        imp = np.ascontiguousarray(store.imp[job.base][:job.n].numpy())
        k = synth.keep_counts(job.n, job.ratios)
        kept = orc.prune_select(imp, k)
        want = orc.quant_sweep(attr, imp, kept, k, G, bits)
        b = mgs.search(job.n, C, k, G, bits, want["err"], want["bits"], 8 * job.budget_bytes)
        r = by_id[job.job_id]
        assert r.best_t == b["best_t"] >= 0, job.job_id
        assert np.array_equal(r.best_bits, b["best_bits"]), job.job_id
        offs = np.concatenate([[0], np.cumsum(k)])
        kt = kept[offs[r.best_t]:offs[r.best_t + 1]]
        oc, _, _ = orc.quantize(attr, kt, G, b["best_bits"])
        assert np.array_equal(r.codes, oc), job.job_id


def test_search_streamed_equals_search(torch):
    """mgs_search_streamed, started while the tables are still being copied
    ratio by ratio (copy stream, one event per ratio, in the order the search
    reads them), returns exactly what mgs_search returns on the finished
    copy: the medium workload's GPU tables."""
    w = synth.workload("medium")
    a, i = w.make()
    attr, imp = dev(torch, a), dev(torch, i)
    k = w.k
    kept = mgs.prune_select(imp, k)
    tab = mgs.quant_sweep(attr, imp, kept, k, w.group, w.bits)
    torch.cuda.synchronize()
    T = len(k)
    budget = w.n * w.channels * 32 // 30
    want = mgs.search(w.n, w.channels, k, w.group, w.bits, host(tab["err"]), host(tab["bits"]), budget)
    err_h = torch.empty(tab["err"].shape, dtype=torch.float64, pin_memory=True)
    bits_h = torch.empty(tab["bits"].shape, dtype=torch.float64, pin_memory=True)
    err_h.fill_(np.nan)
    bits_h.fill_(np.nan)
    cs = torch.cuda.Stream()
    events = [torch.cuda.Event() for _ in range(T)]
    order = [0] + list(range(T - 1, 0, -1))  # increasing k first, then decreasing
    with torch.cuda.stream(cs):
        for t in order:
            err_h[t].copy_(tab["err"][t], non_blocking=True)
            bits_h[t].copy_(tab["bits"][t], non_blocking=True)
            events[t].record(cs)
    got = mgs.search(w.n, w.channels, k, w.group, w.bits, err_h.numpy(), bits_h.numpy(), budget,
                     events=events)
    torch.cuda.synchronize()
    assert got["best_t"] == want["best_t"]
    assert np.array_equal(got["best_bits"], want["best_bits"])
    assert np.array_equal(got["status"], want["status"])
    assert np.array_equal(got["used"], want["used"])
    assert np.array_equal(got["obj"], want["obj"], equal_nan=True)
