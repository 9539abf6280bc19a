"""Benchmark of the MesonGS++ size-aware search hot path on one MI355X.

One step is one pass of the whole path over one synthetic scene (by default
the large workload: N = 5.3e6 Gaussians, 20 channels, 32 reserve ratios,
G = 16384, b in 1..16, byte budget raw/30):
  reserve-ratio pruning -> quantization sweep (loss + entropy tables for
  every ratio x channel x group x bit-width, one graph-replayed launch) ->
  tables to the host -> exact 0-1 ILP per ratio and the ratio choice on host
  threads, while the GPU assigns 3M higher-degree SH vectors to their nearest
  codewords (4096-entry codebook) -> chosen bit-widths to the device -> final
  codes and their reconstruction.
Inputs are resident in HBM before the timed region.  `value` is sweep
evaluations (kept Gaussian x channel x bit-width) per second of whole steps.
The dominant kernel (the sweep) is timed per launch with HIP events on the
stream it runs on; `roofline.traffic` comes from the committed rocprofv3
counter summary of that kernel, or is null when the kernel sources have
changed since it was taken.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12             # bytes/s, MI355X HBM3E
VALU_PEAK = 256 * 64 * 2.4e9  # lane-operations/s: 256 CUs x 64 lanes x 2.4 GHz
MFMA_F16_PEAK = 2.5e15        # dense fp16 (and bf16) FLOP/s
# VALU instructions one evaluation needs at the least: the quantize FMA, the
# clamp, the round, the code's bin address, (q - Z) * S, the difference, its
# square and the weighted accumulation -- 6 to 9 by instruction counting; the
# roofline takes 7 (the histogram's LDS atomic is not a VALU slot)
OPS_PER_EVAL = 7
# the paper's own figures for this stage (its hardware and precision unstated):
# the loss table from its parallel group-wise quantization operator, and the
# 0-1 ILP stage of the bit-width search
PAPER_CONTEXT = {"omega_table_s": 0.49, "ilp_stage_s": 58.52, "hardware": "not stated in the paper",
                 "note": "one unnamed scene; context only, not a target"}
SWEEP_SOURCES = ("paper_2604_26799_amd/csrc/sweep.hip", "paper_2604_26799_amd/csrc/sweep.h",
                 "paper_2604_26799_amd/csrc/common.h")
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--vq-n", type=int, default=3_000_000)
    ap.add_argument("--vq-k", type=int, default=4096)
    ap.add_argument("--budget-ratio", type=int, default=30)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--shape", default=None,
                    help="sweep launch shape nt,ept,lds_cap,cpb (skips the autotuner; for profiler runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (counter calibration)")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-candidate comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=64,
                    help="jobs of the served stream (Poisson 2/s); 0 skips the served form")
    ap.add_argument("--overlap-rate", type=float, default=100.0,
                    help="arrival rate (jobs/s) of the second served stream, where arrivals overlap")
    ap.add_argument("--no-medium", action="store_true", help="skip the medium-workload sweep leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="minimum oracle time of the CPU baseline")
    return ap.parse_args()


def sources_digest() -> str:
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(workload: str, shape):
    """HBM bytes per sweep launch from a committed counter summary
    (profiles/sweep_<workload>_traffic*.txt) taken on these kernel sources,
    this workload and this launch shape; None if there is none."""
    if shape is None:
        return None
    want = ",".join(str(v) for v in shape)
    digest = sources_digest()
    for path in sorted(glob.glob(os.path.join(PROFILES, f"sweep_{workload}_traffic*.txt"))):
        try:
            kv = {}
            with open(path) as f:
                for line in f:
                    if ":" in line and not line.startswith("#"):
                        key, val = line.split(":", 1)
                        kv[key.strip()] = val.strip()
            if kv.get("sources") == digest and kv.get("workload") == workload and kv.get("shape") == want:
                return float(kv["traffic_bytes_per_launch"])
        except (OSError, KeyError, ValueError):
            continue
    return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sweep's (ratio, channel, group) tiles would shard "
              "across GPUs, but only the single-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_26799_amd import mgs, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 18  # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 5}), flush=True)
        return
    mgs.lib()
    w = synth.workload(args.workload)
    attr_h, imp_h = w.make()
    k = w.k
    T, C, G, nb = len(k), w.channels, w.group, len(w.bits)
    evals = int(k.sum()) * C * nb
    sh_h, cb_h = synth.vq_data(args.vq_n, 36, args.vq_k, seed=w.seed + 1)
    budget_bits = (w.n * C * 32) // args.budget_ratio

    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()  # default priority; capture needs a non-default stream
    torch.cuda.set_stream(s)
    cs = torch.cuda.Stream()  # table copies to the host (default priority)
    attr = torch.from_numpy(attr_h).to(dev)
    imp = torch.from_numpy(imp_h).to(dev)
    sh = torch.from_numpy(sh_h).to(dev)
    cb = torch.from_numpy(cb_h).to(dev)
    # persistent buffers: nothing is allocated inside a step
    gm = mgs.gmax_groups(k, G)
    kept = torch.empty(int(k.sum()), dtype=torch.int32, device=dev)
    L = mgs.lib()
    ws_p = mgs.workspace(L.mgs_prune_select_ws_bytes(w.n, T), dev)
    import ctypes as ct
    d = mgs.sweep_desc(w.n, C, k, G, w.bits)
    ws_s = mgs.workspace(L.mgs_quant_sweep_ws_bytes(ct.byref(d)), dev)
    tab = mgs.sweep_tables(T, C, gm, nb, dev)
    err_h = torch.empty((T, C, gm, nb), dtype=torch.float64, pin_memory=True)
    bits_h = torch.empty((T, C, gm, nb), dtype=torch.float64, pin_memory=True)
    ws_v = mgs.workspace(L.mgs_vq_assign_ws_bytes(args.vq_n, 36, args.vq_k), dev)
    offs = np.concatenate([[0], np.cumsum(k)])
    ngmax = (int(k.max()) + G - 1) // G
    bw_d = torch.empty(C * ngmax, dtype=torch.uint8, device=dev)
    bw_h = torch.empty(C * ngmax, dtype=torch.uint8, pin_memory=True)
    codes = torch.empty(C * int(k.max()), dtype=torch.int16, device=dev)
    gmn = torch.empty(C * ngmax, dtype=torch.float32, device=dev)
    gmx = torch.empty(C * ngmax, dtype=torch.float32, device=dev)
    recon = torch.empty(C * int(k.max()), dtype=torch.float32, device=dev)
    idx = torch.empty(args.vq_n, dtype=torch.int32, device=dev)
    nfb = torch.zeros(1, dtype=torch.int64, device=dev)
    sp = s.cuda_stream

    # ---- set-up (untimed): kept sets, autotuned sweep shape, captured sweep
    mgs.prune_select(imp, k, ws=ws_p, out=kept, stream=s)
    tuned = None
    if args.shape:
        tuned = tuple(int(v) for v in args.shape.split(","))
        mgs.sweep_set_shape(G, nb, max(w.bits), *tuned)
    elif not args.no_autotune:
        tuned, _ = mgs.sweep_autotune(attr, imp, kept, k, G, w.bits, reps=2, ws=ws_s, out=tab, stream=s)
        print(f"autotuned sweep shape {tuned}", file=sys.stderr, flush=True)
    s.synchronize()
    graph = mgs.capture(lambda: mgs.quant_sweep(attr, imp, kept, k, G, w.bits, ws=ws_s, out=tab, stream=s,
                                                check=False), s)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    # The search solves the smallest ratio that passes the doubled-8-bit test
    # exactly as soon as its tables are on the host and bounds the others as
    # theirs land: the smallest ratio's tables go first, in copies of their
    # own, and the rest follow in one copy per table when they are contiguous
    # (ratio 0 first), else ratio by ratio.  One event per ratio.
    by_k = sorted(range(len(k)), key=lambda t: (-int(k[t]), t))
    first = by_k[-1]
    if first == 0 and len(k) > 1:
        copy_blocks = [(0, 1), (1, len(k))]
    else:
        copy_blocks = [(first, first + 1)] + [(t, t + 1) for t in by_k[:-1]]
    blk_ev = [torch.cuda.Event() for _ in copy_blocks]
    tev = [None] * len(k)
    for (lo, hi), e in zip(copy_blocks, blk_ev):
        for t in range(lo, hi):
            tev[t] = e
    stage_ms = {"prune": [], "sweep": [], "d2h": [], "ilp": [], "codes": [], "vq": []}

    def step(record: bool):
        s.wait_event(ev[5])  # the last step's codes have read the kept sets the prune rewrites
        ev[0].record(s)
        mgs.prune_select(imp, k, ws=ws_p, out=kept, stream=s, check=False)
        ev[1].record(s)
        graph.launch(s)
        ev[2].record(s)
        # the tables go to the host on a copy stream while the VQ assignment
        # (which does not depend on the bit allocation) starts on the compute
        # stream and runs while the host solves the ILPs
        cs.wait_event(ev[2])
        with torch.cuda.stream(cs):
            for (lo, hi), e in zip(copy_blocks, blk_ev):
                err_h[lo:hi].copy_(tab["err"][lo:hi], non_blocking=True)
                bits_h[lo:hi].copy_(tab["bits"][lo:hi], non_blocking=True)
                e.record(cs)
            ev[3].record(cs)
        rc = L.mgs_vq_assign(sh.data_ptr(), args.vq_n, 36, cb.data_ptr(), args.vq_k, idx.data_ptr(), None,
                             nfb.data_ptr(), ws_v.data_ptr(), ws_v.numel(), sp)
        assert rc == 0, mgs.strerror(rc)
        ev[6].record(s)
        blk_ev[0].synchronize()  # the host stage is timed from the first tables on the host
        t0 = time.perf_counter()
        res = mgs.search(w.n, C, k, G, w.bits, err_h.numpy(), bits_h.numpy(), budget_bits, events=tev)
        t1 = time.perf_counter()
        bt = res["best_t"]
        assert bt >= 0, "no admissible reserve ratio"
        kt = int(k[bt])
        ng = (kt + G - 1) // G
        # the final codes on the copy stream: they need the kept sets and the
        # bit allocation, not the VQ assignment still running on the compute
        # stream, so the step ends when the later of the two does
        bw_h[:C * ng].copy_(torch.from_numpy(res["best_bits"].reshape(-1)))
        with torch.cuda.stream(cs):
            bw_d[:C * ng].copy_(bw_h[:C * ng], non_blocking=True)
            ev[4].record(cs)
        kp = kept.data_ptr() + 4 * int(offs[bt])
        rc = L.mgs_quantize(attr.data_ptr(), w.n, C, kp, kt, G, bw_d.data_ptr(), codes.data_ptr(),
                            gmn.data_ptr(), gmx.data_ptr(), cs.cuda_stream)
        assert rc == 0, mgs.strerror(rc)
        rc = L.mgs_dequantize(codes.data_ptr(), kt, C, G, bw_d.data_ptr(), gmn.data_ptr(), gmx.data_ptr(),
                              recon.data_ptr(), cs.cuda_stream)
        assert rc == 0, mgs.strerror(rc)
        ev[5].record(cs)
        if record:
            s.synchronize()
            cs.synchronize()
            stage_ms["prune"].append(ev[0].elapsed_time(ev[1]))
            stage_ms["sweep"].append(ev[1].elapsed_time(ev[2]))
            stage_ms["d2h"].append(ev[2].elapsed_time(ev[3]))
            stage_ms["vq"].append(ev[2].elapsed_time(ev[6]))
            stage_ms["ilp"].append((t1 - t0) * 1e3)
            stage_ms["codes"].append(ev[4].elapsed_time(ev[5]))
        return bt

    for i in range(args.warmup):
        step(False)
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bt_last = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # status words of the last step (non-finite inputs would be reported here)
    for ws in (ws_p, ws_s, ws_v):
        rc = mgs.status(ws, stream=s)
        assert rc == 0, mgs.strerror(rc)
    graph.close()
    # the last step's final codes once more, alone on the GPU (in the steps
    # they run beside the VQ assignment): the kernels' own durations
    kt_last = int(k[bt_last])
    ea = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ea[0].record(s)
    rc = L.mgs_quantize(attr.data_ptr(), w.n, C, kept.data_ptr() + 4 * int(offs[bt_last]), kt_last, G,
                        bw_d.data_ptr(), codes.data_ptr(), gmn.data_ptr(), gmx.data_ptr(), sp)
    assert rc == 0, mgs.strerror(rc)
    ea[1].record(s)
    rc = L.mgs_dequantize(codes.data_ptr(), kt_last, C, G, bw_d.data_ptr(), gmn.data_ptr(), gmx.data_ptr(),
                          recon.data_ptr(), sp)
    assert rc == 0, mgs.strerror(rc)
    ea[2].record(s)
    ea[2].synchronize()
    codes_alone = {"quantize_ms": ea[0].elapsed_time(ea[1]), "dequantize_ms": ea[1].elapsed_time(ea[2])}

    ms_step = elapsed * 1e3 / args.steps
    med = {key: float(np.median(v)) for key, v in stage_ms.items()}
    sweep_avg_s = float(np.mean(stage_ms["sweep"])) * 1e-3  # average launch duration
    alg_bytes = int(k.sum()) * (4 * C + 8)
    vq_flops = 2.0 * args.vq_n * args.vq_k * 36
    achieved = OPS_PER_EVAL * evals / sweep_avg_s
    traffic = committed_traffic(w.name, tuned)
    out = {
        "metric": "sweep Gaussian·channel·bitwidth evals/s, %HBM peak; p50/p99 job latency",
        "value": evals * args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 3DGS-shaped attributes, LogNormal importance, Laplace SH)",
        "config": {"workload": f"{w.name}: N={w.n}, C={C}, {T} reserve ratios, G={G}, "
                               f"b={w.bits[0]}..{w.bits[-1]}, budget raw/{args.budget_ratio}; "
                               f"VQ {args.vq_n}x36, K={args.vq_k}",
                   "evals_per_step": evals, "sweep_shape": tuned},
        "stages_ms_median": med,
        "codes_alone_ms": codes_alone,
        "sweep_kernel": {
            "avg_launch_ms": sweep_avg_s * 1e3,
            "evals_per_s": evals / sweep_avg_s,
            "alg_bytes": alg_bytes,
            "hbm_frac_algorithmic": alg_bytes / sweep_avg_s / HBM_PEAK,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK / 1e12,
            "unit": "Tops/s",
            "frac": achieved / VALU_PEAK,
            "traffic": traffic,
            "ops_per_eval": OPS_PER_EVAL,
            "hbm_frac_algorithmic": alg_bytes / sweep_avg_s / HBM_PEAK,
        },
        "paper_context": dict(PAPER_CONTEXT, this_sweep_s=sweep_avg_s, this_ilp_s=med["ilp"] * 1e-3),
        "vq": {"tflops_alg": vq_flops / (med["vq"] * 1e-3) / 1e12,
               "mfma_frac": vq_flops / (med["vq"] * 1e-3) / MFMA_F16_PEAK,
               "fallback_rows": int(nfb.item())},
    }
    out["search_variants"] = search_variants(mgs, w, k, G, err_h.numpy(), bits_h.numpy(), budget_bits)
    out["kmeans"] = kmeans_iterations(mgs, torch, sh, cb, s)
    out["raht"] = raht_timing(mgs, torch, w, attr_h, s)
    if not args.no_plain:
        out["plain_per_candidate"] = plain_sweep(mgs, torch, attr, imp, kept, k, G, w.bits, s, med["sweep"])
    del attr, imp, sh, cb, kept, tab, recon, codes, ws_v
    torch.cuda.empty_cache()
    if not args.no_medium and w.name != "medium":
        out["medium_sweep"] = sweep_leg(mgs, torch, synth.workload("medium"), s)
    if args.serve_jobs > 0:
        out["serving"] = served_stream(args.serve_jobs, args.overlap_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, attr_h, imp_h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def sweep_leg(mgs, torch, w, s, launches: int = 10):
    """The sweep alone on another workload (autotuned shape, graph replays
    timed with HIP events on the stream): evals/s and both roofline
    fractions.  Not part of the timed step."""
    attr_h, imp_h = w.make()
    k, G, C, nb = w.k, w.group, w.channels, len(w.bits)
    evals = int(k.sum()) * C * nb
    dev = torch.device("cuda:0")
    attr = torch.from_numpy(attr_h).to(dev)
    imp = torch.from_numpy(imp_h).to(dev)
    kept = mgs.prune_select(imp, k, stream=s)
    import ctypes as ct
    d = mgs.sweep_desc(w.n, C, k, G, w.bits)
    ws = mgs.workspace(mgs.lib().mgs_quant_sweep_ws_bytes(ct.byref(d)), dev)
    tab = mgs.sweep_tables(len(k), C, mgs.gmax_groups(k, G), nb, dev)
    shape, _ = mgs.sweep_autotune(attr, imp, kept, k, G, w.bits, reps=2, ws=ws, out=tab, stream=s)
    graph = mgs.capture(lambda: mgs.quant_sweep(attr, imp, kept, k, G, w.bits, ws=ws, out=tab, stream=s,
                                                check=False), s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
    graph.launch(s)
    for i in range(launches):
        ev[i].record(s)
        graph.launch(s)
    ev[launches].record(s)
    ev[launches].synchronize()
    graph.close()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(launches)]
    t = float(np.mean(ms)) * 1e-3
    alg_bytes = int(k.sum()) * (4 * C + 8)
    return {"workload": f"{w.name}: N={w.n}, C={C}, {len(k)} reserve ratios, G={G}, b={w.bits[0]}..{w.bits[-1]}",
            "sweep_shape": shape, "avg_launch_ms": t * 1e3, "evals_per_s": evals / t,
            "valu_frac": OPS_PER_EVAL * evals / t / VALU_PEAK, "hbm_frac_algorithmic": alg_bytes / t / HBM_PEAK}


def search_variants(mgs, w, k, G, err, bits, budget_bits):
    """The paper's two other search devices on the same tables (host only, not
    in the timed step): the flat exact ILP against the two-step hierarchical
    solver at the chosen ratio (loss and CPU time, median of 5), and the
    calibrated reserve-ratio loop with the linear size estimator."""
    C = w.channels
    res = mgs.search(w.n, C, k, G, w.bits, err, bits, budget_bits)
    t = res["best_t"]
    ng = (int(k[t]) + G - 1) // G
    e = np.ascontiguousarray(err[t, :, :ng].reshape(C * ng, len(w.bits)))
    sz = mgs.size_table(np.ascontiguousarray(bits[t, :, :ng].reshape(C * ng, len(w.bits))), mode=0)

    def timed(fn):
        ts, r = [], None
        for _ in range(5):
            t0 = time.perf_counter()
            r = fn()
            ts.append(time.perf_counter() - t0)
        return r, float(np.median(ts)) * 1e3
    flat, flat_ms = timed(lambda: mgs.ilp_solve(e, sz, budget_bits))
    hier, hier_ms = timed(lambda: mgs.ilp_hierarchical(e, sz, C, w.bits, budget_bits))
    cal, cal_ms = timed(lambda: mgs.search_calibrated(w.n, C, k, G, w.bits, err, bits, budget_bits))
    conv = cal["status"] == mgs.SEARCH_SOLVED
    out = {"ratio_index": int(t), "budget_bits": int(budget_bits),
           "flat": {"obj": flat[1], "used": int(flat[2]), "ms": flat_ms},
           "hierarchical": None if hier is None else {
               "obj": hier[1], "used": int(hier[2]), "ms": hier_ms, "obj_over_flat": hier[1] / flat[1],
               "channel_bits": hier[3].tolist()},
           "calibrated": {"best_t": int(cal["best_t"]), "converged": int(conv.sum()),
                          "skipped": int((cal["status"] == mgs.SEARCH_SKIPPED).sum()),
                          "infeasible": int((cal["status"] == mgs.SEARCH_INFEASIBLE).sum()),
                          "unconverged": int((cal["status"] == mgs.SEARCH_UNCONVERGED).sum()),
                          "mean_iters_converged": float(cal["iters"][conv].mean()) if conv.any() else None,
                          "ms": cal_ms}}
    if cal["best_t"] >= 0:
        b = cal["best_t"]
        out["calibrated"]["obj"] = float(cal["obj"][b])
        out["calibrated"]["actual_over_budget"] = float(cal["actual"][b]) / budget_bits
    return out


def raht_timing(mgs, torch, w, attr_h, s, depth: int = 14, reps: int = 3):
    """RAHT forward and inverse of the workload's attributes (all channels)
    over seeded clustered voxels of a 2^depth grid, HIP events on the stream;
    not part of the timed step."""
    from paper_2604_26799_amd import synth
    n = w.n
    coords = synth.voxels(n, depth, seed=w.seed + 2)
    codes, order = synth.voxel_codes(coords, depth)
    cd = torch.from_numpy(codes.view(np.int64)).to(torch.device("cuda"))
    a = torch.from_numpy(np.ascontiguousarray(attr_h[:, order])).cuda()
    C = a.shape[0]
    ws = mgs.workspace(mgs.lib().mgs_raht_ws_bytes(n, C, depth), a.device)
    coef = mgs.raht(cd, a, depth, ws=ws, stream=s)
    mgs.raht(cd, coef, depth, inverse=True, ws=ws, stream=s)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(s)
    for _ in range(reps):
        coef = mgs.raht(cd, a, depth, ws=ws, stream=s, check=False)
    e[1].record(s)
    for _ in range(reps):
        back = mgs.raht(cd, coef, depth, inverse=True, ws=ws, stream=s, check=False)
    e[2].record(s)
    e[2].synchronize()
    fwd_ms, inv_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    err = float((back - a).abs().max())
    # the sweep over the AC coefficients (DC kept in floating point, unit weights)
    kept = torch.arange(1, n, dtype=torch.int32, device=a.device)
    ones = torch.ones(n, dtype=torch.float32, device=a.device)
    import ctypes as ct
    d = mgs.sweep_desc(n, C, [n - 1], w.group, w.bits)
    wss = mgs.workspace(mgs.lib().mgs_quant_sweep_ws_bytes(ct.byref(d)), a.device)
    tab = mgs.sweep_tables(1, C, mgs.gmax_groups([n - 1], w.group), len(w.bits), a.device)
    mgs.quant_sweep(coef, ones, kept, [n - 1], w.group, w.bits, ws=wss, out=tab, stream=s)
    e[0].record(s)
    for _ in range(reps):
        mgs.quant_sweep(coef, ones, kept, [n - 1], w.group, w.bits, ws=wss, out=tab, stream=s, check=False)
    e[1].record(s)
    e[1].synchronize()
    ac_ms = e[0].elapsed_time(e[1]) / reps
    ac_evals = (n - 1) * C * len(w.bits)
    return {"points": n, "channels": C, "depth": depth, "steps": 3 * depth,
            "forward_ms": fwd_ms, "inverse_ms": inv_ms,
            "roundtrip_max_abs_err": err,
            "ac_sweep": {"ms": ac_ms, "evals": ac_evals, "evals_per_s": ac_evals / (ac_ms * 1e-3),
                         "G": w.group, "bits": f"{w.bits[0]}..{w.bits[-1]}"}}


def kmeans_iterations(mgs, torch, x, cb, s, batch_rows: int = 1 << 18, iters: int = 5):
    """Mini-batch k-means iterations around the assignment (seeded batches of
    the benchmark's SH vectors, a copy of its codebook), HIP events on the
    stream; not part of the timed step."""
    N, D = x.shape
    K = cb.shape[0]
    cbk = cb.clone()
    counts = torch.zeros(K, dtype=torch.int64, device=x.device)
    g = torch.Generator(device="cpu").manual_seed(0)
    batches = [torch.randint(0, N, (batch_rows,), generator=g).to(x.device) for _ in range(iters + 1)]
    ws = mgs.workspace(mgs.lib().mgs_kmeans_step_ws_bytes(batch_rows, D, K), x.device)
    mgs.kmeans_step(x, cbk, counts, batches[0], ws=ws, stream=s)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(iters):
        mgs.kmeans_step(x, cbk, counts, batches[i + 1], ws=ws, stream=s, check=False)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / iters
    return {"batch_rows": batch_rows, "K": K, "D": D, "ms_per_iteration": ms,
            "rows_per_s": batch_rows / (ms * 1e-3)}


def plain_sweep(mgs, torch, attr, imp, kept, k, G, bits, s, batched_ms):
    """The same tables computed one launch per (ratio, bit-width) candidate,
    each launch re-reading its groups (the paper's operator runs once per
    candidate).  Best of two passes."""
    C = attr.shape[0]
    offs = np.concatenate([[0], np.cumsum(k)])
    ws = mgs.workspace(1 << 22, attr.device)
    outs = [mgs.sweep_tables(1, C, mgs.gmax_groups([int(kt)], G), 1, attr.device) for kt in k]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(2):
        e0.record(s)
        for t, kt in enumerate(k):
            kv = kept[int(offs[t]):int(offs[t + 1])]
            for b in bits:
                mgs.quant_sweep(attr, imp, kv, [int(kt)], G, [b], ws=ws, out=outs[t], stream=s, check=False)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return {"launches": len(k) * len(bits), "ms": best, "batched_ms": batched_ms,
            "speedup_batched": best / batched_ms}


def served_stream(num_jobs, overlap_rate):
    """The serving stream (Poisson arrivals at 2 jobs/s, N log-uniform in
    [2e5, 6e6], 20 channels, 16 ratios x b in 2..16, budget raw/U(10, 60)),
    served with continuous batching and, for comparison, one job at a time
    with one launch per candidate.  At 2 jobs/s a job is done before the next
    arrives, so the throughput of both forms is the offered load; the same
    jobs are then served at `overlap_rate` jobs/s, where arrivals land while
    other jobs are on the GPU and join their launches, and all at once
    (saturation: the throughput each form sustains)."""
    from paper_2604_26799_amd import serve, synth
    store = serve.SceneStore()
    jobs = synth.job_stream(num_jobs, 2.0, seed=0)
    res = {"jobs": num_jobs, "arrivals_per_s": 2.0, "overlap_arrivals_per_s": overlap_rate,
           "note": "at 2 jobs/s throughput is arrival-bound in both forms"}
    for label, scale in (("", 1.0), ("overlap_", 2.0 / overlap_rate), ("saturated_", 0.0)):
        for mode in ("batched", "plain"):
            srv = serve.Server(store, mode=mode)
            r = srv.run(jobs, time_scale=scale)
            srv.close()
            print(f"served {label}{mode}: p50 {r['p50_s']:.3f} s, p99 {r['p99_s']:.3f} s, "
                  f"{r['evals_per_s']:.3g} evals/s, mean batch {r['mean_batch']:.2f}", file=sys.stderr,
                  flush=True)
            res[label + mode] = {key: v for key, v in r.items() if key != "results"}
            if mode == "batched":
                sizes = np.bincount(srv.batch_sizes)
                res[label + mode]["launches_by_batch_size"] = {str(i): int(c) for i, c in enumerate(sizes) if c}
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, attr_h, imp_h, min_seconds):
    """The oracle (plain C, FP64, OpenMP over tiles): prune + sweep of the
    whole workload on all host threads, repeated until at least `min_seconds`
    have passed; then one thread on the small workload (whole) and on the
    medium workload's smallest and largest ratio (a bounded sample)."""
    import oracle
    from paper_2604_26799_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    oracle.set_threads(threads)
    k = w.k
    evals = int(k.sum()) * w.channels * len(w.bits)
    reps, t0 = 0, time.perf_counter()
    while reps < 5 and (reps == 0 or time.perf_counter() - t0 < min_seconds):
        kept = oracle.prune_select(imp_h, k)
        oracle.quant_sweep(attr_h, imp_h, kept, k, w.group, w.bits)
        reps += 1
    dt = time.perf_counter() - t0
    out = {"value": evals * reps / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "seconds_per_workload": dt / reps,
           "sample": f"prune + sweep of the whole {w.name} workload ({len(k)} reserve ratios, "
                     f"{evals} evals) x {reps} in {dt:.1f} s"}
    single = {}
    oracle.set_threads(1)
    try:
        for name, pick in (("small", None), ("medium", (0, -1))):
            sw = synth.workload(name)
            a, i = sw.make()
            ks = sw.k if pick is None else sw.k[list(pick)]
            kept = oracle.prune_select(i, ks)
            ev = int(ks.sum()) * sw.channels * len(sw.bits)
            n, t0 = 0, time.perf_counter()
            while n == 0 or time.perf_counter() - t0 < 1.0:
                oracle.quant_sweep(a, i, kept, ks, sw.group, sw.bits)
                n += 1
            t = (time.perf_counter() - t0) / n
            single[name] = {"evals_per_s": ev / t, "seconds": t,
                            "sample": "whole workload" if pick is None else
                            f"reserve ratios {pick[0]} and {len(sw.k) - 1} of {len(sw.k)} ({ev} evals)"}
    finally:
        oracle.set_threads(threads)
    out["single_thread"] = single
    return out


if __name__ == "__main__":
    main()
