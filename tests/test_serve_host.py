"""Host-side pieces of the served form (no GPU): admission by memory, the
device footprint of a job, and the job stream."""
import numpy as np

from paper_2604_26799_amd import serve, synth


def test_admission_caps_resident_bytes():
    a = serve.Admission(100)
    assert a.try_admit(60)
    assert a.try_admit(40)
    assert not a.try_admit(1)          # would exceed the cap
    a.release(60)
    assert a.try_admit(50)
    assert not a.try_admit(20)
    a.release(40)
    a.release(50)
    assert a.used == 0 and a.resident == 0


def test_admission_lets_an_oversized_job_run_alone():
    a = serve.Admission(100)
    assert a.try_admit(500)             # nothing resident: admitted despite the cap
    assert not a.try_admit(1)
    a.release(500)
    assert a.try_admit(1)


def test_plain_mode_admission_is_one_job_at_a_time():
    a = serve.Admission(0)
    assert a.try_admit(10)
    assert not a.try_admit(10)
    a.release(10)
    assert a.try_admit(10)


def test_job_device_bytes_grows_with_the_scene():
    G, nb = 8192, 15
    ratios = synth.ratios_uniform(synth.Fraction(1, 5), synth.Fraction(19, 20), 16)
    prev = 0
    for n in (200_000, 1_000_000, 6_000_000):
        k = synth.keep_counts(n, ratios)
        b = serve.job_device_bytes(n, k, G, nb)
        assert b > 84 * n + 4 * int(k.sum())  # inputs and kept sets at least
        assert b > prev
        prev = b


def test_job_stream_shape():
    jobs = synth.job_stream(64, 2.0, seed=0)
    arr = np.array([j.arrival_s for j in jobs])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    assert 10 < arr[-1] < 70                        # 63 gaps of mean 0.5 s
    ns = np.array([j.n for j in jobs])
    assert ns.min() >= 200_000 and ns.max() <= synth.BASE_N
    ratio = np.array([80 * j.n / j.budget_bytes for j in jobs])
    assert ratio.min() >= 10 - 1e-6 and ratio.max() <= 60 + 1e-3
    assert {j.base for j in jobs} == set(range(synth.NUM_BASES))
    assert all(len(j.ratios) == 16 for j in jobs)
