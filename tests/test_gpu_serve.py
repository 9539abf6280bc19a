"""Served form on the GPU: each job's result (chosen ratio, bit-widths and
final codes) is the same when it runs alone and when it shares launches with
other jobs, and the final codes equal the oracle's at the chosen allocation."""
import numpy as np
import pytest

from paper_2604_26799_amd import serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def store():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return serve.SceneStore(num_bases=2, n=300_000)


def test_served_results_same_alone_and_in_mix(store, orc):
    jobs = synth.job_stream(8, 2.0, seed=3, n_lo=20_000, n_hi=300_000)
    srv = serve.Server(store, mode="batched", mem_cap_bytes=160 << 20, keep_codes=True)
    mix = srv.run(jobs, time_scale=0.002)   # all eight arrive within ~10 ms
    srv.close()
    print({k: v for k, v in mix.items() if k != "results"}, flush=True)
    assert mix["jobs"] == 8
    assert mix["max_batch"] >= 2            # launches were shared
    by_id = {r.job_id: r for r in mix["results"]}
    for job in jobs:
        one = serve.Server(store, mode="batched", keep_codes=True)
        alone = one.run([job], time_scale=0.0)["results"][0]
        one.close()
        r = by_id[job.job_id]
        assert r.best_t == alone.best_t >= 0, job.job_id
        assert np.array_equal(r.best_bits, alone.best_bits), job.job_id
        assert np.array_equal(r.codes, alone.codes), job.job_id
    # final codes of one job against the oracle at the chosen allocation
    job = jobs[0]
    r = by_id[job.job_id]
    attr = store.attr[job.base][:, :job.n].numpy()
    imp = store.imp[job.base][:job.n].numpy()
    k = synth.keep_counts(job.n, job.ratios)
    kept = orc.prune_select(imp, k)
    offs = np.concatenate([[0], np.cumsum(k)])
    kt = kept[offs[r.best_t]:offs[r.best_t + 1]]
    want, _, _ = orc.quantize(np.ascontiguousarray(attr), kt, 8192, r.best_bits)
    assert np.array_equal(r.codes, want)


def test_plain_mode_serves_every_job(store):
    jobs = synth.job_stream(3, 2.0, seed=4, n_lo=20_000, n_hi=100_000)
    srv = serve.Server(store, mode="plain", keep_codes=True)
    out = srv.run(jobs, time_scale=0.0)
    srv.close()
    assert out["jobs"] == 3 and out["max_batch"] == 1
    assert out["launches"] == sum(len(j.ratios) for j in jobs) * 15
    for r in out["results"]:
        assert r.best_t >= 0 and r.codes.shape[0] == 20
        assert set(np.unique(r.best_bits)) <= set(range(2, 17))


def test_nonfinite_job_fails_alone(store):
    """A job whose scene holds a NaN fails with ENONFINITE; the stream goes on
    and the other jobs of the same launch get the results they get on clean
    data (the flagged launch is swept again one job per launch)."""
    from paper_2604_26799_amd import mgs
    bad = serve.SceneStore(num_bases=2, n=100_000)
    bad.attr[1][3, 10] = float("nan")        # every job on base 1 sees it (n > 10)
    jobs = synth.job_stream(6, 2.0, seed=5, n_lo=20_000, n_hi=100_000)
    srv = serve.Server(bad, mode="batched", keep_codes=True)
    out = srv.run(jobs, time_scale=0.0)       # all six in one launch
    srv.close()
    clean = serve.SceneStore(num_bases=2, n=100_000)
    ref_srv = serve.Server(clean, mode="batched", keep_codes=True)
    ref = {r.job_id: r for r in ref_srv.run(jobs, time_scale=0.0)["results"]}
    ref_srv.close()
    assert out["jobs"] == 6 and out["failed"] == 3
    for r in out["results"]:
        if jobs[r.job_id].base == 1:
            assert r.status == mgs.ENONFINITE and r.best_t == -1 and r.best_bits is None
        else:
            assert r.status == mgs.OK and r.best_t == ref[r.job_id].best_t >= 0
            assert np.array_equal(r.best_bits, ref[r.job_id].best_bits)
            assert np.array_equal(r.codes, ref[r.job_id].codes)
