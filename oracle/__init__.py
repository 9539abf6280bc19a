"""CPU oracle for the MesonGS++ quantization sweep -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product library never does.  It shares no
code with the HIP path; the two meet only through the seeded inputs of
``paper_2604_26799_amd.synth``.

Everything here is the plain definition written out (C in ``mgs_oracle.c``,
FP64 accumulation, literal FP32 quantizer), wrapped with NumPy arrays.
Error codes: 0 ok, -1 invalid argument, -2 non-finite input, -3 infeasible.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, EINVAL, ENONFINITE, EINFEASIBLE = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libmgs_oracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        _LIB = ct.CDLL(path)
        P = ct.c_void_p
        i64, i32 = ct.c_int64, ct.c_int32
        _LIB.orc_prune_select.argtypes = [P, i64, P, i32, P]
        _LIB.orc_quant_sweep.argtypes = [P, i64, i32, i64, P, P, P, i32, i32, P, i32, P, P, P, P, P]
        _LIB.orc_quantize.argtypes = [P, i64, i32, i64, P, i64, i32, P, P, P, P]
        _LIB.orc_dequantize.argtypes = [P, i64, i32, i32, P, P, P, P]
        _LIB.orc_vq_assign.argtypes = [P, i64, i32, P, i32, P, P]
        _LIB.orc_ilp_exhaustive.argtypes = [P, P, i64, i32, i64, P, P, P]
        _LIB.orc_ilp_dp.argtypes = [P, P, i64, i32, i64, P, P, P]
        _LIB.orc_hist_bins.argtypes = [P, i32]
        _LIB.orc_hist_bins.restype = i64
        for f in ("orc_prune_select", "orc_quant_sweep", "orc_quantize", "orc_dequantize",
                  "orc_vq_assign", "orc_ilp_exhaustive", "orc_ilp_dp"):
            getattr(_LIB, f).restype = ct.c_int
    return _LIB


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops for later calls from this thread
    (libgomp's omp_set_num_threads); returns the number in effect before."""
    lib()
    gomp = ct.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = ct.c_int
    before = int(gomp.omp_get_max_threads())
    gomp.omp_set_num_threads(ct.c_int(int(n)))
    return before


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _check(code: int, what: str, allow=(OK,)):
    if code not in allow:
        raise OracleError(code, what)
    return code


def prune_select(imp: np.ndarray, k) -> np.ndarray:
    """Kept indices per reserve ratio, concatenated (each ascending)."""
    imp = np.ascontiguousarray(imp, dtype=np.float32)
    k = np.ascontiguousarray(k, dtype=np.int64)
    out = np.empty(int(k.sum()), dtype=np.int32)
    _check(lib().orc_prune_select(_p(imp), imp.size, _p(k), k.size, _p(out)), "prune_select")
    return out


def gmax_groups(k, G: int) -> int:
    return int((int(np.max(k)) + G - 1) // G)


def quant_sweep(attr: np.ndarray, imp: np.ndarray, kept: np.ndarray, k, G: int, bits,
                want_hist: bool = False):
    """Loss / size tables ``err, bits [T][C][Gmax][nb]`` and ``gmin, gmax [T][C][Gmax]``.

    Returns a dict; with ``want_hist`` also ``hist [T][C][Gmax][sum 2^b]``.
    Raises OracleError on invalid or non-finite input.
    """
    attr = np.ascontiguousarray(attr, dtype=np.float32)
    C, N = attr.shape
    imp = np.ascontiguousarray(imp, dtype=np.float32)
    kept = np.ascontiguousarray(kept, dtype=np.int32)
    k = np.ascontiguousarray(k, dtype=np.int64)
    bl = np.ascontiguousarray(bits, dtype=np.uint8)
    T, nb = k.size, bl.size
    gm = gmax_groups(k, G) if k.size else 0
    err = np.empty((T, C, gm, nb), dtype=np.float64)
    bt = np.empty((T, C, gm, nb), dtype=np.float64)
    mn = np.empty((T, C, gm), dtype=np.float32)
    mx = np.empty((T, C, gm), dtype=np.float32)
    hist = None
    hp = None
    if want_hist:
        hb = int(lib().orc_hist_bins(_p(bl), nb))
        hist = np.empty((T, C, gm, hb), dtype=np.uint32)
        hp = _p(hist)
    _check(lib().orc_quant_sweep(_p(attr), N, C, N, _p(imp), _p(kept), _p(k), T, G, _p(bl), nb,
                                 _p(err), _p(bt), _p(mn), _p(mx), hp), "quant_sweep")
    return {"err": err, "bits": bt, "gmin": mn, "gmax": mx, "hist": hist}


def quantize(attr: np.ndarray, kept: np.ndarray, G: int, bw: np.ndarray):
    """Codes ``u16[C][k]`` and ``gmin, gmax [C][ceil(k/G)]`` at bit-widths ``bw[C][ng]``."""
    attr = np.ascontiguousarray(attr, dtype=np.float32)
    C, N = attr.shape
    kept = np.ascontiguousarray(kept, dtype=np.int32)
    k = kept.size
    ng = (k + G - 1) // G
    bw = np.ascontiguousarray(bw, dtype=np.uint8).reshape(C, ng)
    codes = np.empty((C, k), dtype=np.uint16)
    mn = np.empty((C, ng), dtype=np.float32)
    mx = np.empty((C, ng), dtype=np.float32)
    _check(lib().orc_quantize(_p(attr), N, C, N, _p(kept), k, G, _p(bw), _p(codes), _p(mn), _p(mx)),
           "quantize")
    return codes, mn, mx


def dequantize(codes: np.ndarray, G: int, bw: np.ndarray, gmin: np.ndarray, gmax: np.ndarray):
    codes = np.ascontiguousarray(codes, dtype=np.uint16)
    C, k = codes.shape
    out = np.empty((C, k), dtype=np.float32)
    _check(lib().orc_dequantize(_p(codes), k, C, G, _p(np.ascontiguousarray(bw, dtype=np.uint8)),
                                _p(np.ascontiguousarray(gmin, dtype=np.float32)),
                                _p(np.ascontiguousarray(gmax, dtype=np.float32)), _p(out)),
           "dequantize")
    return out


def vq_assign(x: np.ndarray, cb: np.ndarray):
    """``(idx i32[n], dist f64[n])``: nearest codeword, FP64 distances, ties -> lowest index."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    cb = np.ascontiguousarray(cb, dtype=np.float32)
    n, D = x.shape
    K = cb.shape[0]
    idx = np.empty(n, dtype=np.int32)
    dist = np.empty(n, dtype=np.float64)
    _check(lib().orc_vq_assign(_p(x), n, D, _p(cb), K, _p(idx), _p(dist)), "vq_assign")
    return idx, dist


def _ilp(fn, err, size, budget):
    err = np.ascontiguousarray(err, dtype=np.float64)
    size = np.ascontiguousarray(size, dtype=np.int64)
    ncls, nopt = err.shape
    choice = np.empty(ncls, dtype=np.uint8)
    obj = ct.c_double(0.0)
    used = ct.c_int64(0)
    code = fn(_p(err), _p(size), ncls, nopt, int(budget), _p(choice), ct.byref(obj), ct.byref(used))
    _check(code, "ilp", allow=(OK, EINFEASIBLE))
    if code == EINFEASIBLE:
        return None
    return choice, obj.value, used.value


def ilp_exhaustive(err, size, budget):
    """Exact 0-1 ILP by enumeration (<= 8 classes).  None if infeasible."""
    return _ilp(lib().orc_ilp_exhaustive, err, size, budget)


def ilp_dp(err, size, budget):
    """Exact 0-1 ILP by dynamic programming over the integer budget.  None if infeasible."""
    return _ilp(lib().orc_ilp_dp, err, size, budget)


METADATA_BITS = 72  # per group: FP32 minimum + FP32 maximum + one byte of bit-width


def size_table(bits_table: np.ndarray, n_per_group=None, bit_list=None, mode: str = "entropy"):
    """Integer ILP sizes per (group, option): ceil(entropy bits) + 72, or n*b + 72."""
    if mode == "entropy":
        return np.ceil(bits_table).astype(np.int64) + METADATA_BITS
    if mode == "linear":
        n = np.asarray(n_per_group, dtype=np.int64)[:, None]
        b = np.asarray(bit_list, dtype=np.int64)[None, :]
        return n * b + METADATA_BITS
    raise ValueError(mode)


def choose_ratio(per_tau):
    """Reserve-ratio choice of the search, one plain reading of its outer loop.

    ``per_tau``: list of dicts with keys ``tau`` (comparable), ``size8`` (bits of
    the all-8-bit configuration), ``budget`` (bits), ``obj`` (ILP optimum or None
    if infeasible).  A ratio whose doubled 8-bit size is below the budget is
    skipped; among the rest with a feasible ILP the smallest loss wins; a tie
    goes to the larger ratio.  Returns the index into ``per_tau`` or None.
    """
    best = None
    for i, r in enumerate(per_tau):
        if 2 * r["size8"] < r["budget"]:
            continue
        if r["obj"] is None:
            continue
        if best is None or r["obj"] < per_tau[best]["obj"] or (
                r["obj"] == per_tau[best]["obj"] and r["tau"] > per_tau[best]["tau"]):
            best = i
    return best


def ilp_hierarchical(err, size, C: int, bit_list, budget: int, solve=None):
    """The two-step solver of section "Solve the MINLP", paragraph
    "Hierarchical Solver": first one bit-width per channel (every group of the
    channel at that option; the channel's loss and size are the sums over its
    groups, added in group order), solved exactly under the whole budget
    S_T; then the channel budgets S_c = floor(S_T * Q_c / sum_c Q_c) and, per
    channel, the exact group-level ILP within S_c.

    Classes are C channels x ng groups, channel-major.  Returns (choice, obj,
    used, chan_bits, chan_budget) or None when a step has no feasible
    allocation.  ``solve`` is the exact solver (default: ``ilp_dp``).
    """
    solve = solve or ilp_dp
    err = np.asarray(err, dtype=np.float64)
    size = np.asarray(size, dtype=np.int64)
    ncls, nopt = err.shape
    ng = ncls // C
    assert ng * C == ncls
    ec = np.zeros((C, nopt), dtype=np.float64)
    sc = np.zeros((C, nopt), dtype=np.int64)
    for c in range(C):
        for g in range(ng):
            for j in range(nopt):
                ec[c, j] += err[c * ng + g, j]
                sc[c, j] += size[c * ng + g, j]
    top = solve(ec, sc, budget)
    if top is None:
        return None
    q = [int(bit_list[j]) for j in top[0]]
    qsum = sum(q)
    choice = np.empty(ncls, dtype=np.uint8)
    obj, used, shares = 0.0, 0, []
    for c in range(C):
        share = (int(budget) * q[c]) // qsum
        r = solve(err[c * ng:(c + 1) * ng], size[c * ng:(c + 1) * ng], share)
        if r is None:
            return None
        choice[c * ng:(c + 1) * ng] = r[0]
        obj += r[1]
        used += r[2]
        shares.append(share)
    return choice, obj, used, np.array(q, dtype=np.uint8), np.array(shares, dtype=np.int64)


SOLVED, SKIPPED, INFEASIBLE, UNCONVERGED = 0, 1, 2, 4


def search_calibrated(err_tab, bits_tab, k, G: int, bit_list, budget: int, tol_ppm: int = 50000,
                      max_iter: int = 16, solve=None):
    """Algorithm 1 "Hyperparameter Optimization" with the size estimator of
    equation "size_estim" (linear: n * b bits per group + 72 metadata bits +
    S_delta) and the entropy table as the measured size (ceil(bits) + 72 per
    group).

    Per ratio t, in the algorithm's order: start from every group at 8 bits
    and measure it (n * 8 + 72 per group when 8 is not a candidate); skip the
    ratio when twice that size is below the budget S_T; then repeat: S_delta =
    measured size - linear estimate of the current allocation, solve the ILP
    with linear sizes and the constraint estimate + S_delta <= S_T, measure
    the new allocation, and stop when |S_a - S_T| / S_T < tol (integer test
    |S_a - S_T| * 10^6 < tol_ppm * S_T), at most ``max_iter`` solves.  The
    kept ratio is the converged one with the smallest loss (ties: larger k,
    then larger index).

    ``err_tab`` / ``bits_tab``: [T][C][Gmax][nb] tables.  Returns dict(best_t,
    best_bits [C][ng] or None, and per ratio obj, actual, iters, status).
    """
    solve = solve or ilp_dp
    err_tab = np.asarray(err_tab, dtype=np.float64)
    bits_tab = np.asarray(bits_tab, dtype=np.float64)
    T, C, _, nb = err_tab.shape
    bl = [int(b) for b in bit_list]
    i8 = bl.index(8) if 8 in bl else None
    obj = np.full(T, np.nan)
    actual = np.zeros(T, dtype=np.int64)
    iters = np.zeros(T, dtype=np.int32)
    status = np.full(T, UNCONVERGED, dtype=np.int32)
    choices = [None] * T
    for t in range(T):
        kt = int(k[t])
        ng = (kt + G - 1) // G
        if ng == 0:
            status[t] = SKIPPED
            continue
        e = err_tab[t, :, :ng].reshape(C * ng, nb)
        b = bits_tab[t, :, :ng].reshape(C * ng, nb)
        n = np.tile([min(G, kt - g * G) for g in range(ng)], C)
        act = size_table(b, mode="entropy")
        lin = size_table(b, n, bl, "linear")
        sa = sum(int(act[i, i8]) if i8 is not None else int(n[i]) * 8 + METADATA_BITS for i in range(C * ng))
        est = sum(int(n[i]) * 8 + METADATA_BITS for i in range(C * ng))
        actual[t] = sa
        if 2 * sa < budget:
            status[t] = SKIPPED
            continue
        for it in range(1, max_iter + 1):
            delta = sa - est
            limit = budget - delta
            r = solve(e, lin, limit) if limit >= 0 else None
            if r is None:
                status[t] = INFEASIBLE
                break
            choice, o, used = r
            sa = sum(int(act[i, choice[i]]) for i in range(C * ng))
            est = int(used)
            obj[t], actual[t], iters[t], choices[t] = o, sa, it, choice
            if abs(sa - budget) * 1000000 < tol_ppm * budget:
                status[t] = SOLVED
                break
    best = None
    for t in range(T):
        if status[t] != SOLVED:
            continue
        if best is None or obj[t] < obj[best] or (obj[t] == obj[best] and (k[t] > k[best] or (
                k[t] == k[best] and t > best))):
            best = t
    best_bits = None
    if best is not None:
        ng = (int(k[best]) + G - 1) // G
        best_bits = np.array([bl[j] for j in choices[best]], dtype=np.uint8).reshape(C, ng)
    return {"best_t": -1 if best is None else best, "best_bits": best_bits, "obj": obj, "actual": actual,
            "iters": iters, "status": status}


def kmeans_step(x, cb, counts, batch):
    """One iteration of the batched clustering the paper uses for the
    higher-degree SH vectors (section "Attribute Transformation", paragraph
    "Clustering 1+D SH Coefficients", citing Sculley's web-scale k-means):
    the batch rows are first all assigned to their nearest center (the exact
    FP64 rule of ``vq_assign``, against the centers before this iteration),
    then taken in batch order, each moving its center with the per-center
    learning rate 1 / v:  v_j += 1,  c_j <- (1 - 1/v_j) c_j + (1/v_j) x  (FP64).
    The updated centers are stored as FP32.  Returns (centers f32 [K][D],
    counts i64 [K], assignment i32 [B]).
    """
    x = np.asarray(x, dtype=np.float32)
    cb = np.asarray(cb, dtype=np.float32)
    batch = np.asarray(batch, dtype=np.int64)
    rows = x[batch]
    assign, _ = vq_assign(np.ascontiguousarray(rows), cb)
    c = cb.astype(np.float64)
    v = np.array(counts, dtype=np.int64).copy()
    for r in range(batch.size):
        j = int(assign[r])
        v[j] += 1
        eta = 1.0 / float(v[j])
        c[j] = (1.0 - eta) * c[j] + eta * rows[r].astype(np.float64)
    return c.astype(np.float32), v, assign


def kmeans_step_batched(x, cb, counts, batch):
    """The same iteration in the batched form of the running mean (section
    "Attribute Transformation", paragraph "Clustering 1+D SH Coefficients"):
    the batch rows are assigned to their nearest center (``vq_assign``), then
    every center j with n_j > 0 rows moves to
        c_j <- (v_j c_j + S_j) / (v_j + n_j),   v_j += n_j,
    where S_j is the FP64 sum of its rows taken one after another in batch
    order, and the products, sums and quotient are single FP64 operations in
    that order; the center is stored as FP32.  Returns (centers f32 [K][D],
    counts i64 [K], assignment i32 [B])."""
    x = np.asarray(x, dtype=np.float32)
    cb = np.asarray(cb, dtype=np.float32)
    batch = np.asarray(batch, dtype=np.int64)
    rows = x[batch]
    assign, _ = vq_assign(np.ascontiguousarray(rows), cb)
    out = cb.copy()
    v = np.array(counts, dtype=np.int64).copy()
    for j in range(cb.shape[0]):
        mine = rows[assign == j].astype(np.float64)
        n = mine.shape[0]
        if n == 0:
            continue
        total = np.zeros(cb.shape[1], dtype=np.float64)
        for r in range(n):           # one row after another, in batch order
            total = total + mine[r]
        vj = np.float64(v[j])
        out[j] = ((vj * cb[j].astype(np.float64) + total) / np.float64(v[j] + n)).astype(np.float32)
        v[j] += n
    return out, v, assign


def vq_retain(x, imp, cb, idx, remaining_bits: int):
    """Budget-first retention (same paragraph of the paper): with the bits
    left after the essential components, keep the original vectors of the
    most important Gaussians -- r = min(N, floor(remaining / (32 D))) of
    them, D FP32 values each -- append them to the codebook in ascending
    Gaussian index and point their index entries at them.  Returns (extended
    codebook, new index table, r)."""
    x = np.asarray(x, dtype=np.float32)
    N, D = x.shape
    r = 0 if remaining_bits <= 0 else min(N, int(remaining_bits) // (32 * D))
    idx = np.array(idx, dtype=np.int32).copy()
    if r == 0:
        return np.asarray(cb, dtype=np.float32).copy(), idx, 0
    top = prune_select(np.asarray(imp, dtype=np.float32), [r])
    K = cb.shape[0]
    ext = np.concatenate([np.asarray(cb, dtype=np.float32), x[top]], axis=0)
    idx[top] = K + np.arange(r, dtype=np.int32)
    return ext, idx, r


def morton(coords, depth: int) -> np.ndarray:
    """Morton code of integer voxel coordinates: bit 3l of the code is bit l
    of x, bit 3l+1 of y, bit 3l+2 of z."""
    coords = np.asarray(coords, dtype=np.int64)
    code = np.zeros(coords.shape[0], dtype=np.uint64)
    for l in range(depth):
        for a in range(3):
            code |= ((coords[:, a] >> l) & 1).astype(np.uint64) << np.uint64(3 * l + a)
    return code


def raht_forward(coords, attr, depth: int):
    """RAHT (section "Attribute Transformation", paragraph "Region Adaptive
    Hierarchical Transform"): per level from the finest, along x, then y, then
    z, every two occupied nodes that differ only in the current axis' bit are
    merged by T_1 with their weights (leaves 1, merged nodes the sum); the
    first output goes up, the second is an AC coefficient; unmatched nodes go
    up unchanged.  Nodes are kept in Morton order (the order of the input,
    which must be sorted by it), so ACs come out step by step in that order.
    FP64 as  L = (s1 a1 + s2 a2) / s,  H = (s1 a2 - s2 a1) / s,
    s1 = sqrt(w1), s2 = sqrt(w2), s = sqrt(w1 + w2).
    Returns the coefficients f32 [C][N]: DC first, then the ACs.
    """
    coords = np.asarray(coords, dtype=np.int64)
    attr = np.asarray(attr, dtype=np.float32)
    codes = morton(coords, depth)
    assert np.all(np.diff(codes.astype(np.float64)) > 0) and np.all(codes[1:] > codes[:-1])
    C, N = attr.shape
    nodes = [[tuple(coords[i]), 1, attr[:, i].astype(np.float64)] for i in range(N)]
    acs = []
    for level in range(depth):
        for axis in range(3):
            new = []
            i = 0
            while i < len(nodes):
                pos, w1, a1 = nodes[i]
                up = list(pos)
                up[axis] >>= 1
                up = tuple(up)
                if pos[axis] & 1 == 0 and i + 1 < len(nodes):
                    pos2, w2, a2 = nodes[i + 1]
                    up2 = list(pos2)
                    up2[axis] >>= 1
                    if tuple(up2) == up:
                        s1, s2, sw = np.sqrt(float(w1)), np.sqrt(float(w2)), np.sqrt(float(w1 + w2))
                        acs.append((s1 * a2 - s2 * a1) / sw)
                        new.append([up, w1 + w2, (s1 * a1 + s2 * a2) / sw])
                        i += 2
                        continue
                new.append([up, w1, a1])
                i += 1
            nodes = new
    assert len(nodes) == 1
    out = np.empty((C, N), dtype=np.float32)
    out[:, 0] = nodes[0][2]
    for j, h in enumerate(acs):
        out[:, 1 + j] = h
    return out
