"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments before touching the device (runs without a GPU)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2604_26799_amd import mgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "mgs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mgs_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = mgs.lib()
    syms = header_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(mgs.SIGNATURES), "binding and header disagree"


def test_strerror_and_version():
    assert mgs.strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5, -6):
        assert mgs.strerror(code) not in ("ok", "unknown status")
    assert b"gfx950" in mgs.lib().mgs_version()


def test_sweep_rejects_bad_descriptors():
    L = mgs.lib()
    fake = ct.c_void_p(0x1000)  # never dereferenced: validation fails first
    base = dict(N=100, C=2, k=[50, 100], G=16, bits=[2, 4])

    def call(**kw):
        a = dict(base)
        a.update(kw)
        d = mgs.sweep_desc(a["N"], a["C"], a["k"], a["G"], a["bits"])
        if "ld" in kw:
            d.ld = kw["ld"]
        return L.mgs_quant_sweep(ct.byref(d), fake, fake, fake, fake, fake, fake, fake, None, None, 0, None)

    assert call(G=0) == mgs.EINVAL
    assert call(G=65536) == mgs.EINVAL
    assert call(bits=[4, 2]) == mgs.EINVAL          # not increasing
    assert call(bits=[2, 2]) == mgs.EINVAL          # duplicate
    assert call(bits=[0, 3]) == mgs.EINVAL
    assert call(bits=[3, 17]) == mgs.EINVAL
    assert call(k=[101]) == mgs.EINVAL              # k > N
    assert call(k=[-1]) == mgs.EINVAL
    assert call(k=[1] * 65) == mgs.EINVAL           # too many ratios
    assert call(ld=50) == mgs.EINVAL                # ld < N
    assert call() == mgs.EWORKSPACE                 # valid, but no workspace
    assert L.mgs_quant_sweep(None, fake, fake, fake, fake, fake, fake, fake, None, fake, 1 << 20,
                             None) == mgs.EINVAL


def test_multi_sweep_rejects_bad_job_lists():
    L = mgs.lib()
    fake = 0x1000
    jobs = (mgs.SweepJob * 2)()
    keep = []
    for i, G in enumerate((16, 32)):
        d = mgs.sweep_desc(100, 2, [50], G, [2, 4])
        keep.append(d)
        jobs[i].desc = d
        for f in ("d_attr", "d_imp", "d_kept", "d_err", "d_bits", "d_gmin", "d_gmax"):
            setattr(jobs[i], f, fake)
    ws = ct.c_void_p(fake)
    assert L.mgs_quant_sweep_multi(jobs, 0, ws, 1 << 30, None) == mgs.EINVAL
    assert L.mgs_quant_sweep_multi(jobs, 65, ws, 1 << 30, None) == mgs.EINVAL
    assert L.mgs_quant_sweep_multi(None, 1, ws, 1 << 30, None) == mgs.EINVAL
    assert L.mgs_quant_sweep_multi(jobs, 2, ws, 1 << 30, None) == mgs.EINVAL   # G differs
    jobs[1].desc = keep[0]
    jobs[1].d_err = None
    assert L.mgs_quant_sweep_multi(jobs, 2, ws, 1 << 30, None) == mgs.EINVAL   # missing table
    jobs[1].d_err = fake
    assert L.mgs_quant_sweep_multi(jobs, 2, None, 0, None) == mgs.EWORKSPACE
    assert L.mgs_quant_sweep_multi_ws_bytes(jobs, 2) > L.mgs_quant_sweep_multi_ws_bytes(jobs, 1) > 0


def test_host_solvers_reject_bad_arguments():
    L = mgs.lib()
    P = lambda a: a.ctypes.data_as(ct.c_void_p)
    err = np.zeros((4, 2))
    size = np.full((4, 2), 5, np.int64)
    ch = np.zeros(4, np.uint8)
    o, u = ct.c_double(), ct.c_int64()
    bl = np.array([2, 4], np.uint8)

    def hier(*, e=err, C=2, ng=2, nopt=2, bits=bl, budget=100):
        return L.mgs_ilp_hierarchical(P(e) if e is not None else None, P(size), C, ng, nopt, P(bits), budget,
                                      P(ch), ct.byref(o), ct.byref(u), None, None)
    assert hier() == mgs.OK
    assert hier(bits=np.array([0, 4], np.uint8)) == mgs.EINVAL  # bit-width 0
    assert hier(C=0) == mgs.EINVAL
    assert hier(budget=-1) == mgs.EINVAL
    assert hier(e=None) == mgs.EINVAL
    assert hier(e=np.full((4, 2), np.nan)) == mgs.EINVAL
    assert hier(budget=5) == mgs.EINFEASIBLE
    d = mgs.sweep_desc(20, 1, [20], 10, [4, 8])
    tab = np.zeros((1, 1, 2, 2))
    bt, ob = ct.c_int32(), np.zeros(2, np.uint8)
    outs = [np.zeros(1), np.zeros(1, np.int64), np.zeros(1, np.int32), np.zeros(1, np.int32)]

    def calib(budget=100, tol=50000, iters=4):
        return L.mgs_search_calibrated(ct.byref(d), P(tab), P(tab), budget, tol, iters, 1, ct.byref(bt), P(ob),
                                       *[P(x) for x in outs])
    assert calib() in (mgs.OK, mgs.EINFEASIBLE)
    assert calib(budget=0) == mgs.EINVAL
    assert calib(tol=-1) == mgs.EINVAL
    assert calib(tol=1000001) == mgs.EINVAL
    assert calib(iters=0) == mgs.EINVAL

    # the streamed search checks its events before it waits for any
    res = [np.zeros(1), np.zeros(1, np.int64), np.zeros(1, np.int32)]

    def streamed(events):
        return L.mgs_search_streamed(ct.byref(d), P(tab), P(tab), 100, 0, 1, 0, ct.byref(bt), P(ob),
                                     *[P(x) for x in res], events)
    assert streamed(None) == mgs.EINVAL
    assert streamed((ct.c_void_p * 1)(None)) == mgs.EINVAL


def test_graph_calls_reject_null_handles():
    L = mgs.lib()
    h = ct.c_void_p()
    assert L.mgs_graph_begin(None) == mgs.EINVAL
    assert L.mgs_graph_end(None, ct.byref(h)) == mgs.EINVAL
    assert L.mgs_graph_launch(None, None) == mgs.EINVAL
    assert L.mgs_graph_destroy(None) == mgs.EINVAL


def test_other_entry_points_reject_bad_arguments():
    L = mgs.lib()
    fake = ct.c_void_p(0x1000)
    k = np.array([5], np.int64)
    kp = k.ctypes.data_as(ct.c_void_p)
    assert L.mgs_prune_select(None, 10, kp, 1, fake, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_prune_select(fake, 10, kp, 0, fake, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_prune_select(fake, 4, kp, 1, fake, fake, 1 << 20, None) == mgs.EINVAL  # k > n
    assert L.mgs_prune_select(fake, 10, kp, 1, fake, None, 0, None) == mgs.EWORKSPACE
    assert L.mgs_quantize(fake, 10, 0, fake, 5, 4, fake, fake, fake, fake, None) == mgs.EINVAL
    assert L.mgs_quantize(fake, 10, 2, fake, 5, 0, fake, fake, fake, fake, None) == mgs.EINVAL
    assert L.mgs_quantize(fake, 10, 2, None, 5, 4, fake, fake, fake, fake, None) == mgs.EINVAL
    assert L.mgs_dequantize(fake, 5, 2, 70000, fake, fake, fake, fake, None) == mgs.EINVAL
    assert L.mgs_vq_assign(fake, 10, 0, fake, 4, fake, None, None, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_vq_assign(fake, 10, 65, fake, 4, fake, None, None, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_vq_assign(fake, 10, 36, fake, 0, fake, None, None, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_vq_assign(fake, 10, 36, fake, (1 << 30) + 1, fake, None, None, fake, 1 << 20, None) == mgs.EINVAL
    assert L.mgs_vq_assign_ws_bytes(10, 36, (1 << 30) + 1) == 0
    assert L.mgs_vq_assign(fake, 10, 36, fake, 4, fake, None, None, None, 0, None) == mgs.EWORKSPACE
    assert L.mgs_status_fetch(None, None) == mgs.EWORKSPACE


def test_workspace_queries():
    L = mgs.lib()
    assert L.mgs_prune_select_ws_bytes(5_300_000, 32) > L.mgs_prune_select_ws_bytes(1000, 1) > 0
    assert L.mgs_vq_assign_ws_bytes(3_000_000, 36, 4096) >= 3_000_000 * 4
    assert L.mgs_vq_assign_ws_bytes(10, 0, 4) == 0
    d = mgs.sweep_desc(1000, 11, [500, 1000], 4096, [4, 5, 6])
    assert L.mgs_quant_sweep_ws_bytes(ct.byref(d)) >= 256 + 8 * 4097
    # the tile order takes one int per group of a channel run
    small = mgs.sweep_desc(10_000_000, 20, [1_000_000], 1024, [4, 8])
    big = mgs.sweep_desc(10_000_000, 20, [1_000_000] * 8, 1024, [4, 8])
    grow = L.mgs_quant_sweep_ws_bytes(ct.byref(big)) - L.mgs_quant_sweep_ws_bytes(ct.byref(small))
    assert grow >= 4 * 7 * 977 and grow < 4 * 7 * 977 + 512
    # without counts the size bounds every count vector of T ratios over N
    nok = mgs.SweepDesc(10_000_000, 10_000_000, 20, 8, 1024, 2, None, None)
    assert L.mgs_quant_sweep_ws_bytes(ct.byref(nok)) >= 4 * 8 * 9766
    assert L.mgs_quant_sweep_ws_bytes(ct.byref(nok)) >= L.mgs_quant_sweep_ws_bytes(ct.byref(big))


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    """The product path has no fallback: a missing library is an error."""
    monkeypatch.setattr(mgs, "_lib", None)
    monkeypatch.setattr(mgs, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        mgs.lib()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before any device is touched."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_static_sweep_rejects_before_the_device():
    """The allocation-free sweep checks its arguments and its scratch limit
    on the host: a bad descriptor is EINVAL, a launch whose workspace would
    exceed MGS_STATIC_SCRATCH_BYTES (4 MiB; 785,920 groups per channel run at
    G = 65535) is EWORKSPACE -- both without touching a device."""
    L = mgs.lib()
    fake = ct.c_void_p(0x1000)  # never dereferenced: validation fails first

    def call(N, C, k, G, bits):
        d = mgs.sweep_desc(N, C, k, G, bits)
        return L.mgs_quant_sweep_static(ct.byref(d), fake, fake, fake, fake, fake, fake, fake, None, None)

    assert call(100, 2, [50, 100], 0, [2, 4]) == mgs.EINVAL
    assert call(100, 2, [101], 16, [2, 4]) == mgs.EINVAL
    assert call(1_000_000, 2, [1_000_000] * 4, 1, [2, 4]) == mgs.EWORKSPACE
    # the limit is the workspace query against 4 MiB
    for G, groups in ((65535, 785_920), (8192, 1_015_232)):
        for g, fits in ((groups, True), (groups + 1, False)):
            d = mgs.sweep_desc(g * G, 1, [g * G], G, [2])
            assert (L.mgs_quant_sweep_ws_bytes(ct.byref(d)) <= 4 << 20) == fits
    d = mgs.sweep_desc(785_921 * 65535 // 32, 1, [785_921 * 65535 // 32] * 32, 65535, [2])
    assert L.mgs_quant_sweep_static(ct.byref(d), fake, fake, fake, fake, fake, fake, fake, None, None) == mgs.EWORKSPACE
