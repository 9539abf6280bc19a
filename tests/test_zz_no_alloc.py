"""The allocation-free sweep (library scratch array instead of a workspace)
through the C ABI: two calls in a row, the second on a smaller input, each
bit-identical to mgs_quant_sweep with a caller workspace on the same input and
equal to the oracle within the sweep's bar; the status word of the array
follows the last call (a non-finite input raises it, the next clean call
clears it).  Runs alone or after the other tests."""
import ctypes as ct

import numpy as np
import pytest

from paper_2604_26799_amd import mgs, synth

pytestmark = pytest.mark.gpu
ERR_REL = 4e-6


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    mgs.lib()
    return _t


def tables_of(torch, out):
    torch.cuda.synchronize()
    return {key: out[key].cpu().numpy() for key in ("err", "bits", "gmin", "gmax")}


def static_call(torch, attr, imp, kept, k, G, bits, s):
    """mgs_quant_sweep_static straight through the C ABI."""
    C, N = attr.shape
    d = mgs.sweep_desc(N, C, k, G, bits)
    out = mgs.sweep_tables(d.T, C, mgs.gmax_groups(k, G), d.nb, attr.device)
    rc = mgs.lib().mgs_quant_sweep_static(ct.byref(d), attr.data_ptr(), imp.data_ptr(), kept.data_ptr(),
                                          out["err"].data_ptr(), out["bits"].data_ptr(), out["gmin"].data_ptr(),
                                          out["gmax"].data_ptr(), None, s.cuda_stream)
    assert rc == mgs.OK, mgs.strerror(rc)
    return out


@pytest.mark.parametrize("case", ["medium_then_small"])
def test_static_sweep_matches_workspace_sweep(torch, orc, case):
    s = torch.cuda.Stream()
    cases = [(synth.SweepWorkload("a", 400_000, 20, synth.ratios_uniform(synth.Fraction(1, 5),
                                                                         synth.Fraction(19, 20), 8),
                                  8192, list(range(2, 17)), seed=5)),
             synth.workload("small")]
    for w in cases:
        attr_h, imp_h = w.make()
        k = w.k
        print(f"static sweep: {w.name} N={w.n} C={w.channels} T={len(k)} G={w.group}", flush=True)
        attr = torch.from_numpy(attr_h).cuda()
        imp = torch.from_numpy(imp_h).cuda()
        kept = mgs.prune_select(imp, k, stream=s)
        got = tables_of(torch, static_call(torch, attr, imp, kept, k, w.group, w.bits, s))
        assert mgs.lib().mgs_quant_sweep_static_status(s.cuda_stream) == mgs.OK
        ref = tables_of(torch, mgs.quant_sweep(attr, imp, kept, k, w.group, w.bits, stream=s))
        for key in ref:
            assert np.array_equal(got[key], ref[key], equal_nan=True), (w.name, key)
        want = orc.quant_sweep(attr_h, imp_h, kept.cpu().numpy(), k, w.group, w.bits)
        ok = ~np.isnan(want["err"])
        assert np.array_equal(np.isnan(got["err"]), ~ok)
        np.testing.assert_allclose(got["err"][ok], want["err"][ok], rtol=ERR_REL, atol=1e-300)
        np.testing.assert_allclose(got["bits"][ok], want["bits"][ok], rtol=1e-9, atol=1e-6)
        gn = ~np.isnan(want["gmin"])
        assert np.array_equal(got["gmin"][gn], want["gmin"][gn])
        assert np.array_equal(got["gmax"][gn], want["gmax"][gn])


def test_static_sweep_status_word(torch):
    s = torch.cuda.Stream()
    attr_h, imp_h = synth.scene(5000, 11, seed=1)
    k = np.array([5000], np.int64)
    kept = torch.arange(5000, dtype=torch.int32, device="cuda")
    bad = attr_h.copy()
    bad[3, 100] = np.nan
    out = static_call(torch, torch.from_numpy(bad).cuda(), torch.from_numpy(imp_h).cuda(), kept, k, 1024, [4, 8], s)
    assert mgs.lib().mgs_quant_sweep_static_status(s.cuda_stream) == mgs.ENONFINITE
    err = out["err"].cpu().numpy()
    assert np.isnan(err[0, 3, 0]).all() and np.isfinite(err[0, 2]).all()
    # the next clean call starts from a cleared status word
    static_call(torch, torch.from_numpy(attr_h).cuda(), torch.from_numpy(imp_h).cuda(), kept, k, 1024, [4, 8], s)
    assert mgs.lib().mgs_quant_sweep_static_status(s.cuda_stream) == mgs.OK
