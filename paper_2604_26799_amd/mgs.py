"""ctypes binding of libmgs (the C ABI in include/mgs.h).

Argument marshalling only: every step runs in the library (HIP kernels on the
GPU, the 0-1 ILP on the host).  PyTorch supplies device memory and the
current stream.  If the library is missing this module raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgs.so")

OK, EINVAL, ENONFINITE, EINFEASIBLE, EDEVICE, EWORKSPACE, ELIMIT = 0, -1, -2, -3, -4, -5, -6
MAX_RATIOS, MAX_GROUP, MAX_BITS, MAX_VQ_DIM, MAX_JOBS = 64, 65535, 16, 64, 64

_lib = None


class MgsError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class SweepDesc(ct.Structure):
    _fields_ = [("N", ct.c_int64), ("ld", ct.c_int64), ("C", ct.c_int32), ("T", ct.c_int32),
                ("G", ct.c_int32), ("nb", ct.c_int32), ("h_k", ct.c_void_p), ("h_bits", ct.c_void_p)]


class SweepJob(ct.Structure):
    _fields_ = [("desc", SweepDesc), ("d_attr", ct.c_void_p), ("d_imp", ct.c_void_p), ("d_kept", ct.c_void_p),
                ("d_err", ct.c_void_p), ("d_bits", ct.c_void_p), ("d_gmin", ct.c_void_p),
                ("d_gmax", ct.c_void_p), ("d_hist", ct.c_void_p)]


# name -> (restype, argtypes); the full exported surface of include/mgs.h
P, I32, I64, SZ, D = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t, ct.c_double
SIGNATURES = {
    "mgs_strerror": (ct.c_char_p, [ct.c_int]),
    "mgs_version": (ct.c_char_p, []),
    "mgs_status_fetch": (ct.c_int, [P, P]),
    "mgs_prune_select_ws_bytes": (SZ, [I64, I32]),
    "mgs_prune_select": (ct.c_int, [P, I64, P, I32, P, P, SZ, P]),
    "mgs_quant_sweep_ws_bytes": (SZ, [P]),
    "mgs_quant_sweep": (ct.c_int, [P, P, P, P, P, P, P, P, P, P, SZ, P]),
    "mgs_quant_sweep_static": (ct.c_int, [P, P, P, P, P, P, P, P, P, P]),
    "mgs_quant_sweep_static_status": (ct.c_int, [P]),
    "mgs_quant_sweep_multi_ws_bytes": (SZ, [P, I32]),
    "mgs_quant_sweep_multi": (ct.c_int, [P, I32, P, SZ, P]),
    "mgs_sweep_shape_count": (ct.c_int, []),
    "mgs_sweep_autotune": (ct.c_int, [P, P, P, P, P, P, P, P, P, SZ, P, I32, P, P, P]),
    "mgs_sweep_set_shape": (ct.c_int, [I32, I32, I32, I32, I32, I32, I32, I32]),
    "mgs_quantize": (ct.c_int, [P, I64, I32, P, I64, I32, P, P, P, P, P]),
    "mgs_dequantize": (ct.c_int, [P, I64, I32, I32, P, P, P, P, P]),
    "mgs_vq_assign_ws_bytes": (SZ, [I64, I32, I32]),
    "mgs_vq_assign": (ct.c_int, [P, I64, I32, P, I32, P, P, P, P, SZ, P]),
    "mgs_kmeans_step_ws_bytes": (SZ, [I64, I32, I32]),
    "mgs_kmeans_step": (ct.c_int, [P, I64, I32, P, I64, P, I32, P, P, P, SZ, P]),
    "mgs_vq_retain_count": (I64, [I64, I64, I32]),
    "mgs_raht_ws_bytes": (SZ, [I64, I32, I32]),
    "mgs_raht_forward": (ct.c_int, [P, I64, I32, I32, P, I64, P, P, SZ, P]),
    "mgs_raht_inverse": (ct.c_int, [P, I64, I32, I32, P, I64, P, P, SZ, P]),
    "mgs_vq_retain": (ct.c_int, [P, I64, I32, P, I64, P, I32, P, P, SZ, P]),
    "mgs_graph_begin": (ct.c_int, [P]),
    "mgs_graph_end": (ct.c_int, [P, ct.POINTER(ct.c_void_p)]),
    "mgs_graph_launch": (ct.c_int, [P, P]),
    "mgs_graph_destroy": (ct.c_int, [P]),
    "mgs_ilp_solve": (ct.c_int, [P, P, I64, I32, I64, P, P, P]),
    "mgs_size_table": (ct.c_int, [P, P, I64, I32, P, I32, P]),
    "mgs_search": (ct.c_int, [P, P, P, I64, I32, I32, I32, P, P, P, P, P]),
    "mgs_search_streamed": (ct.c_int, [P, P, P, I64, I32, I32, I32, P, P, P, P, P, P]),
    "mgs_ilp_hierarchical": (ct.c_int, [P, P, I32, I64, I32, P, I64, P, P, P, P, P]),
    "mgs_search_calibrated": (ct.c_int, [P, P, P, I64, I32, I32, I32, P, P, P, P, P, P]),
}


def lib():
    """Load libmgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmgs.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().mgs_strerror(code).decode()


def _check(code: int, what: str):
    if code != OK:
        raise MgsError(code, what)


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


# ----------------------------------------------------------------- device side
def _torch():
    import torch
    return torch


def _dptr(t) -> int:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def workspace(nbytes: int, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def status(ws, stream=None) -> int:
    return lib().mgs_status_fetch(_dptr(ws), _stream(stream))


def _finish(ws, check: bool, what: str, stream=None):
    if check:
        code = status(ws, stream)
        if code != OK:
            raise MgsError(code, what)


def prune_select(imp, k: Sequence[int], ws=None, out=None, stream=None, check: bool = True):
    """Kept indices (int32, concatenated per ratio, each ascending) on the device."""
    torch = _torch()
    k = np.ascontiguousarray(k, dtype=np.int64)
    n = imp.numel()
    need = lib().mgs_prune_select_ws_bytes(n, k.size)
    if ws is None or ws.numel() < need:
        ws = workspace(need, imp.device)
    if out is None:
        out = torch.empty(int(k.sum()), dtype=torch.int32, device=imp.device)
    _check(lib().mgs_prune_select(_dptr(imp), n, _np_ptr(k), k.size, _dptr(out) if out.numel() else None,
                                  _dptr(ws), ws.numel(), _stream(stream)), "mgs_prune_select")
    _finish(ws, check, "mgs_prune_select", stream)
    return out


def sweep_desc(N: int, C: int, k, G: int, bits, ld: Optional[int] = None):
    k = np.ascontiguousarray(k, dtype=np.int64)
    bl = np.ascontiguousarray(bits, dtype=np.uint8)
    d = SweepDesc(N, N if ld is None else ld, C, k.size, G, bl.size, k.ctypes.data, bl.ctypes.data)
    d._keep = (k, bl)  # keep the host arrays alive with the descriptor
    return d


def gmax_groups(k, G: int) -> int:
    return int((int(np.max(k)) + G - 1) // G)


def quant_sweep(attr, imp, kept, k, G: int, bits, want_hist: bool = False, ws=None, out=None,
                stream=None, check: bool = True):
    """Loss / size tables ``err, bits [T][C][Gmax][nb]`` (FP64) and ``gmin, gmax`` (FP32)."""
    torch = _torch()
    C, N = attr.shape
    d = sweep_desc(N, C, k, G, bits)
    T, nb = d.T, d.nb
    gm = gmax_groups(k, G)
    dev = attr.device
    need = lib().mgs_quant_sweep_ws_bytes(ct.byref(d))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    if out is None:
        out = {
            "err": torch.empty((T, C, gm, nb), dtype=torch.float64, device=dev),
            "bits": torch.empty((T, C, gm, nb), dtype=torch.float64, device=dev),
            "gmin": torch.empty((T, C, gm), dtype=torch.float32, device=dev),
            "gmax": torch.empty((T, C, gm), dtype=torch.float32, device=dev),
            "hist": None,
        }
        if want_hist:
            hb = int(sum(1 << int(b) for b in d._keep[1]))
            out["hist"] = torch.empty((T, C, gm, hb), dtype=torch.int32, device=dev)
    _check(lib().mgs_quant_sweep(ct.byref(d), _dptr(attr), _dptr(imp), _dptr(kept) if kept.numel() else None,
                                 _dptr(out["err"]), _dptr(out["bits"]), _dptr(out["gmin"]),
                                 _dptr(out["gmax"]), _dptr(out["hist"]), _dptr(ws), ws.numel(),
                                 _stream(stream)), "mgs_quant_sweep")
    _finish(ws, check, "mgs_quant_sweep", stream)
    return out


def quant_sweep_static(attr, imp, kept, k, G: int, bits, out=None, stream=None, check: bool = True):
    """The sweep without a workspace (the library's per-GPU scratch array);
    same tables as ``quant_sweep``."""
    C, N = attr.shape
    d = sweep_desc(N, C, k, G, bits)
    if out is None:
        hb = 0
        out = sweep_tables(d.T, C, gmax_groups(k, G), d.nb, attr.device, hb)
    _check(lib().mgs_quant_sweep_static(ct.byref(d), _dptr(attr), _dptr(imp), _dptr(kept) if kept.numel() else None,
                                        _dptr(out["err"]), _dptr(out["bits"]), _dptr(out["gmin"]),
                                        _dptr(out["gmax"]), _dptr(out.get("hist")), _stream(stream)),
           "mgs_quant_sweep_static")
    if check:
        _check(lib().mgs_quant_sweep_static_status(_stream(stream)), "mgs_quant_sweep_static")
    return out


def sweep_tables(T: int, C: int, gm: int, nb: int, device, hist_bins: int = 0):
    """Empty output tables of one scene's sweep."""
    torch = _torch()
    out = {"err": torch.empty((T, C, gm, nb), dtype=torch.float64, device=device),
           "bits": torch.empty((T, C, gm, nb), dtype=torch.float64, device=device),
           "gmin": torch.empty((T, C, gm), dtype=torch.float32, device=device),
           "gmax": torch.empty((T, C, gm), dtype=torch.float32, device=device),
           "hist": None}
    if hist_bins:
        out["hist"] = torch.empty((T, C, gm, hist_bins), dtype=torch.int32, device=device)
    return out


def sweep_jobs(scenes, G: int, bits, want_hist: bool = False):
    """Job array of a batched sweep.

    ``scenes``: sequence of dicts with ``attr [C][N]`` (or ``[C][ld]`` with ``n``), ``imp``, ``kept``,
    ``k`` and optionally ``out`` (tables, else allocated).  Returns ``(jobs, outs)``.
    """
    n = len(scenes)
    jobs = (SweepJob * n)()
    outs, keep = [], []
    for i, sc in enumerate(scenes):
        attr, imp, kept, k = sc["attr"], sc["imp"], sc["kept"], sc["k"]
        C, ld = attr.shape
        N = int(sc.get("n", ld))
        d = sweep_desc(N, C, k, G, bits, ld=ld)
        gm = gmax_groups(k, G)
        hb = int(sum(1 << int(b) for b in d._keep[1])) if want_hist else 0
        out = sc.get("out") or sweep_tables(d.T, C, gm, d.nb, attr.device, hb)
        jobs[i].desc = d
        jobs[i].d_attr = _dptr(attr)
        jobs[i].d_imp = _dptr(imp)
        jobs[i].d_kept = _dptr(kept) if kept.numel() else None
        for key in ("err", "bits", "gmin", "gmax", "hist"):
            setattr(jobs[i], "d_" + key, _dptr(out[key]))
        outs.append(out)
        keep.append(d)
    jobs._keep = keep  # host arrays referenced by the descriptors
    return jobs, outs


def quant_sweep_multi(scenes, G: int, bits, want_hist: bool = False, ws=None, stream=None, check: bool = True,
                      jobs=None):
    """Batched sweep of several scenes in one launch; returns one table dict per scene."""
    if jobs is None:
        jobs, outs = sweep_jobs(scenes, G, bits, want_hist)
    else:
        outs = None
    n = len(jobs)
    need = lib().mgs_quant_sweep_multi_ws_bytes(jobs, n)
    if ws is None or ws.numel() < need:
        dev = scenes[0]["attr"].device
        ws = workspace(need, dev)
    _check(lib().mgs_quant_sweep_multi(jobs, n, _dptr(ws), ws.numel(), _stream(stream)), "mgs_quant_sweep_multi")
    _finish(ws, check, "mgs_quant_sweep_multi", stream)
    return outs


class Graph:
    """A captured sequence of library calls, replayed with ``launch``."""

    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream=None):
        _check(lib().mgs_graph_launch(self.handle, _stream(stream)), "mgs_graph_launch")

    def close(self):
        if self.handle:
            _check(lib().mgs_graph_destroy(self.handle), "mgs_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture(fn, stream):
    """Record the library calls ``fn()`` makes on ``stream`` (not the default stream) into a Graph."""
    sp = _stream(stream)
    _check(lib().mgs_graph_begin(sp), "mgs_graph_begin")
    try:
        fn()
    except BaseException:
        h = ct.c_void_p()
        lib().mgs_graph_end(sp, ct.byref(h))
        if h.value:
            lib().mgs_graph_destroy(h)
        raise
    h = ct.c_void_p()
    _check(lib().mgs_graph_end(sp, ct.byref(h)), "mgs_graph_end")
    return Graph(h.value)


def sweep_autotune(attr, imp, kept, k, G: int, bits, reps: int = 3, ws=None, out=None, stream=None):
    """Time every launch shape of the sweep on these inputs and register the fastest.

    Returns ``(best (nt, ept, lds_cap, cpb, persist), [(nt, ept, lds_cap, cpb, persist, ms), ...])``.
    """
    torch = _torch()
    C, N = attr.shape
    d = sweep_desc(N, C, k, G, bits)
    T, nb = d.T, d.nb
    gm = gmax_groups(k, G)
    dev = attr.device
    need = lib().mgs_quant_sweep_ws_bytes(ct.byref(d))
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    if out is None:
        out = {"err": torch.empty((T, C, gm, nb), dtype=torch.float64, device=dev),
               "bits": torch.empty((T, C, gm, nb), dtype=torch.float64, device=dev),
               "gmin": torch.empty((T, C, gm), dtype=torch.float32, device=dev),
               "gmax": torch.empty((T, C, gm), dtype=torch.float32, device=dev)}
    n = lib().mgs_sweep_shape_count()
    ms = np.empty(n, dtype=np.float32)
    shapes = np.empty((n, 5), dtype=np.int32)
    best = np.empty(5, dtype=np.int32)
    _check(lib().mgs_sweep_autotune(ct.byref(d), _dptr(attr), _dptr(imp), _dptr(kept), _dptr(out["err"]),
                                    _dptr(out["bits"]), _dptr(out["gmin"]), _dptr(out["gmax"]), _dptr(ws),
                                    ws.numel(), _stream(stream), reps, _np_ptr(ms), _np_ptr(shapes),
                                    _np_ptr(best)), "mgs_sweep_autotune")
    rows = [tuple(int(v) for v in sh) + (float(m),) for sh, m in zip(shapes, ms) if m >= 0]
    return tuple(int(v) for v in best), rows


def sweep_set_shape(G: int, nb: int, bmax: int, nt: int, ept: int, lds_cap: int = 0, cpb: int = 0,
                    persist: int = 0):
    _check(lib().mgs_sweep_set_shape(G, nb, bmax, nt, ept, lds_cap, cpb, persist), "mgs_sweep_set_shape")


def quantize(attr, kept, G: int, bw, stream=None):
    """Codes ``u16 [C][k]`` (returned as int16 storage) and ``gmin, gmax [C][ng]``."""
    torch = _torch()
    C, N = attr.shape
    k = kept.numel()
    ng = (k + G - 1) // G
    dev = attr.device
    codes = torch.empty((C, k), dtype=torch.int16, device=dev)
    mn = torch.empty((C, ng), dtype=torch.float32, device=dev)
    mx = torch.empty((C, ng), dtype=torch.float32, device=dev)
    _check(lib().mgs_quantize(_dptr(attr), N, C, _dptr(kept), k, G, _dptr(bw), _dptr(codes), _dptr(mn),
                              _dptr(mx), _stream(stream)), "mgs_quantize")
    return codes, mn, mx


def dequantize(codes, G: int, bw, gmin, gmax, stream=None):
    torch = _torch()
    C, k = codes.shape
    out = torch.empty((C, k), dtype=torch.float32, device=codes.device)
    _check(lib().mgs_dequantize(_dptr(codes), k, C, G, _dptr(bw), _dptr(gmin), _dptr(gmax), _dptr(out),
                                _stream(stream)), "mgs_dequantize")
    return out


def vq_assign(x, cb, want_dist: bool = True, ws=None, stream=None, check: bool = True):
    """Nearest codeword ``idx i32[N]``, its FP64 distance, and the fallback row count."""
    torch = _torch()
    N, D = x.shape
    K = cb.shape[0]
    dev = x.device
    need = lib().mgs_vq_assign_ws_bytes(N, D, K)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    idx = torch.empty(N, dtype=torch.int32, device=dev)
    dist = torch.empty(N, dtype=torch.float64, device=dev) if want_dist else None
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().mgs_vq_assign(_dptr(x), N, D, _dptr(cb), K, _dptr(idx) if N else None,
                               _dptr(dist) if (dist is not None and N) else None, _dptr(nfb), _dptr(ws),
                               ws.numel(), _stream(stream)), "mgs_vq_assign")
    _finish(ws, check, "mgs_vq_assign", stream)
    return idx, dist, nfb


def kmeans_step(x, cb, counts, batch, ws=None, stream=None, check: bool = True):
    """One mini-batch k-means iteration on the rows ``batch`` (int64) of ``x``:
    ``cb`` (f32 [K][D]) and ``counts`` (i64 [K]) are updated in place; returns the
    batch's assignment ``i32[B]``."""
    torch = _torch()
    N, D = x.shape
    K = cb.shape[0]
    B = batch.numel()
    dev = x.device
    need = lib().mgs_kmeans_step_ws_bytes(B, D, K)
    if ws is None or ws.numel() < need:
        ws = workspace(need, dev)
    assign = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    _check(lib().mgs_kmeans_step(_dptr(x), N, D, _dptr(batch) if B else None, B, _dptr(cb), K, _dptr(counts),
                                 _dptr(assign), _dptr(ws), ws.numel(), _stream(stream)), "mgs_kmeans_step")
    _finish(ws, check, "mgs_kmeans_step", stream)
    return assign[:B]


def vq_retain(x, imp, cb, idx, remaining_bits: int, ws=None, stream=None, check: bool = True):
    """Budget-first retention: the top-r Gaussians by importance (r from the
    remaining bits) keep their own vectors.  Returns (extended codebook
    f32 [K + r][D], r); ``idx`` (i32 [N]) is updated in place."""
    torch = _torch()
    N, D = x.shape
    K = cb.shape[0]
    r = int(lib().mgs_vq_retain_count(int(remaining_bits), N, D))
    cb_ext = torch.empty((K + r, D), dtype=torch.float32, device=x.device)
    cb_ext[:K].copy_(cb)
    if r == 0:
        return cb_ext, 0
    top = prune_select(imp, [r], stream=stream, check=check)
    if ws is None:
        ws = workspace(256, x.device)
    _check(lib().mgs_vq_retain(_dptr(x), N, D, _dptr(top), r, _dptr(cb_ext), K, _dptr(idx), _dptr(ws),
                               ws.numel(), _stream(stream)), "mgs_vq_retain")
    _finish(ws, check, "mgs_vq_retain", stream)
    return cb_ext, r


def raht(codes, values, depth: int, inverse: bool = False, ws=None, stream=None, check: bool = True):
    """RAHT of ``values`` (f32 [C][N], order of the Morton ``codes`` u64/i64 [N])
    or, with ``inverse``, back from coefficients; returns f32 [C][N]."""
    torch = _torch()
    C, N = values.shape
    need = lib().mgs_raht_ws_bytes(N, C, depth)
    if ws is None or ws.numel() < need:
        ws = workspace(need, values.device)
    out = torch.empty((C, N), dtype=torch.float32, device=values.device)
    fn = lib().mgs_raht_inverse if inverse else lib().mgs_raht_forward
    _check(fn(_dptr(codes), N, C, depth, _dptr(values), N, _dptr(out), _dptr(ws), ws.numel(), _stream(stream)),
           "mgs_raht_inverse" if inverse else "mgs_raht_forward")
    _finish(ws, check, "mgs_raht", stream)
    return out


def raht_sweep(codes, attr, depth: int, G: int, bits, ws=None, stream=None, check: bool = True):
    """The quantization sweep over RAHT coefficients (the paper quantizes the AC
    coefficients group-wise and keeps the DC in floating point): RAHT forward of
    ``attr`` (f32 [C][N], Morton order of ``codes``), then one sweep over the
    N - 1 AC columns of every channel, in the order the transform makes them,
    with unit weights (the unweighted squared error).  Returns ``(coef f32
    [C][N], tables)``; the tables have one reserve ratio keeping all N - 1 ACs."""
    torch = _torch()
    C, N = attr.shape
    coef = raht(codes, attr, depth, stream=stream, check=check)
    n_ac = N - 1
    kept = torch.arange(1, N, dtype=torch.int32, device=attr.device)
    ones = torch.ones(N, dtype=torch.float32, device=attr.device)
    tab = quant_sweep(coef, ones, kept, [n_ac], G, bits, ws=ws, stream=stream, check=check)
    return coef, tab


# ----------------------------------------------------------------- host side
def ilp_solve(err: np.ndarray, size: np.ndarray, budget: int):
    """Exact 0-1 ILP; ``(choice u8[ncls], obj, used)`` or None when infeasible."""
    err = np.ascontiguousarray(err, dtype=np.float64)
    size = np.ascontiguousarray(size, dtype=np.int64)
    ncls, nopt = err.shape
    choice = np.empty(ncls, dtype=np.uint8)
    obj = ct.c_double(0.0)
    used = ct.c_int64(0)
    code = lib().mgs_ilp_solve(_np_ptr(err), _np_ptr(size), ncls, nopt, int(budget), _np_ptr(choice),
                               ct.byref(obj), ct.byref(used))
    if code == EINFEASIBLE:
        return None
    _check(code, "mgs_ilp_solve")
    return choice, obj.value, used.value


def size_table(bits_table: np.ndarray, n_per_group=None, bit_list=None, mode: int = 0):
    bits_table = np.ascontiguousarray(bits_table, dtype=np.float64)
    ncls, nb = bits_table.shape
    out = np.empty((ncls, nb), dtype=np.int64)
    n = np.ascontiguousarray(n_per_group if n_per_group is not None else np.zeros(ncls), dtype=np.int64)
    bl = np.ascontiguousarray(bit_list if bit_list is not None else np.zeros(nb), dtype=np.uint8)
    _check(lib().mgs_size_table(_np_ptr(bits_table), _np_ptr(n), ncls, nb, _np_ptr(bl), mode, _np_ptr(out)),
           "mgs_size_table")
    return out


SEARCH_ALL = 1
SEARCH_SOLVED, SEARCH_SKIPPED, SEARCH_INFEASIBLE, SEARCH_PRUNED, SEARCH_UNCONVERGED = 0, 1, 2, 3, 4


def search(N: int, C: int, k, G: int, bits, err: np.ndarray, bits_table: np.ndarray, budget_bits: int,
           size_mode: int = 0, threads: int = 0, solve_all: bool = False, events=None):
    """Reserve-ratio loop + exact ILP over host copies of a sweep's tables.

    Returns dict(best_t, best_bits u8[C][ng], obj f64[T], used i64[T], status i32[T]);
    best_t is -1 when no ratio is admissible.  Without ``solve_all`` ratios whose LP
    bound exceeds the best optimum are not solved (status SEARCH_PRUNED).  With
    ``events`` (one torch.cuda.Event per ratio, recorded after that ratio's table
    slices were copied into ``err`` / ``bits_table``, which must then be the host
    buffers themselves: no copy is made) the search starts while the copies run
    (mgs_search_streamed).
    """
    d = sweep_desc(N, C, k, G, bits)
    if events is not None:
        for a in (err, bits_table):
            if a.dtype != np.float64 or not a.flags.c_contiguous:
                raise ValueError("streamed tables are read in place: contiguous float64 host buffers")
    err = np.ascontiguousarray(err, dtype=np.float64)
    bt = np.ascontiguousarray(bits_table, dtype=np.float64)
    T = d.T
    kk = d._keep[0]
    ngmax = (int(kk.max()) + G - 1) // G
    best_t = ct.c_int32(-1)
    best_bits = np.zeros(C * max(ngmax, 1), dtype=np.uint8)
    obj = np.empty(T, dtype=np.float64)
    used = np.empty(T, dtype=np.int64)
    status = np.empty(T, dtype=np.int32)
    if events is None:
        code = lib().mgs_search(ct.byref(d), _np_ptr(err), _np_ptr(bt), int(budget_bits), size_mode, threads,
                                SEARCH_ALL if solve_all else 0, ct.byref(best_t), _np_ptr(best_bits),
                                _np_ptr(obj), _np_ptr(used), _np_ptr(status))
    else:
        if len(events) != T:
            raise ValueError(f"one event per ratio: {len(events)} events for {T} ratios")
        evs = (ct.c_void_p * T)(*[int(e.cuda_event) for e in events])
        code = lib().mgs_search_streamed(ct.byref(d), _np_ptr(err), _np_ptr(bt), int(budget_bits), size_mode,
                                         threads, SEARCH_ALL if solve_all else 0, ct.byref(best_t),
                                         _np_ptr(best_bits), _np_ptr(obj), _np_ptr(used), _np_ptr(status), evs)
    if code not in (OK, EINFEASIBLE):
        _check(code, "mgs_search")
    t = best_t.value
    ng = (int(kk[t]) + G - 1) // G if t >= 0 else 0
    return {"best_t": t, "best_bits": best_bits[:C * ng].reshape(C, ng) if t >= 0 else None,
            "obj": obj, "used": used, "status": status}


def ilp_hierarchical(err: np.ndarray, size: np.ndarray, C: int, bit_list, budget: int):
    """Two-step (channel, then group) 0-1 ILP over classes C x ng, channel-major.

    Returns (choice u8[C*ng], obj, used, chan_bits u8[C], chan_budget i64[C]), or None
    when a step is infeasible.
    """
    err = np.ascontiguousarray(err, dtype=np.float64)
    size = np.ascontiguousarray(size, dtype=np.int64)
    ncls, nopt = err.shape
    assert ncls % C == 0, "classes must be C channels x ng groups"
    bl = np.ascontiguousarray(bit_list, dtype=np.uint8)
    assert bl.size == nopt
    choice = np.empty(ncls, dtype=np.uint8)
    chan_bits = np.empty(C, dtype=np.uint8)
    chan_budget = np.empty(C, dtype=np.int64)
    obj = ct.c_double(0.0)
    used = ct.c_int64(0)
    code = lib().mgs_ilp_hierarchical(_np_ptr(err), _np_ptr(size), C, ncls // C, nopt, _np_ptr(bl),
                                      int(budget), _np_ptr(choice), ct.byref(obj), ct.byref(used),
                                      _np_ptr(chan_bits), _np_ptr(chan_budget))
    if code == EINFEASIBLE:
        return None
    _check(code, "mgs_ilp_hierarchical")
    return choice, obj.value, used.value, chan_bits, chan_budget


def search_calibrated(N: int, C: int, k, G: int, bits, err: np.ndarray, bits_table: np.ndarray,
                      budget_bits: int, tol_ppm: int = 50000, max_iter: int = 16, threads: int = 0):
    """The calibrated reserve-ratio search (linear size estimator + measured entropy size).

    Returns dict(best_t, best_bits u8[C][ng], obj f64[T], actual i64[T], iters i32[T],
    status i32[T]); best_t is -1 when no ratio converged.
    """
    d = sweep_desc(N, C, k, G, bits)
    err = np.ascontiguousarray(err, dtype=np.float64)
    bt = np.ascontiguousarray(bits_table, dtype=np.float64)
    T = d.T
    kk = d._keep[0]
    ngmax = (int(kk.max()) + G - 1) // G
    best_t = ct.c_int32(-1)
    best_bits = np.zeros(C * max(ngmax, 1), dtype=np.uint8)
    obj = np.empty(T, dtype=np.float64)
    actual = np.empty(T, dtype=np.int64)
    iters = np.empty(T, dtype=np.int32)
    status = np.empty(T, dtype=np.int32)
    code = lib().mgs_search_calibrated(ct.byref(d), _np_ptr(err), _np_ptr(bt), int(budget_bits), int(tol_ppm),
                                       int(max_iter), threads, ct.byref(best_t), _np_ptr(best_bits),
                                       _np_ptr(obj), _np_ptr(actual), _np_ptr(iters), _np_ptr(status))
    if code not in (OK, EINFEASIBLE):
        _check(code, "mgs_search_calibrated")
    t = best_t.value
    ng = (int(kk[t]) + G - 1) // G if t >= 0 else 0
    return {"best_t": t, "best_bits": best_bits[:C * ng].reshape(C, ng) if t >= 0 else None,
            "obj": obj, "actual": actual, "iters": iters, "status": status}
