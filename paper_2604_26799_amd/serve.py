"""Served form of the search: a continuous-batching loop over compression jobs.

A job is a scene (attributes [20][n], importance [n]) plus a byte budget; its
answer is the reserve ratio and per-group bit-widths the search picks and the
final codes at that allocation (paper: Algorithm 1 over the quantization
sweep, section "Acceleration"; the 0-1 ILP of section "Solve the MINLP").

Batched mode (continuous batching):
  * arrivals are admitted while their device footprint fits under a memory
    cap (a job larger than the cap is admitted alone);
  * an admitted job's scene is uploaded on a copy stream, then pruned on the
    compute stream;
  * every device iteration launches ONE multi-scene sweep over all jobs that
    are ready (mgs_quant_sweep_multi); at most `max_inflight` such launches
    are on the GPU at a time, so jobs that become ready while one runs wait
    for it and join the next launch together (iteration-level scheduling);
  * each job's tables come back to pinned host memory and its ILP search runs
    on a host thread pool while the GPU keeps sweeping other jobs;
  * the chosen bit-widths go back, the final codes are quantized on the
    device and copied to the host, and the job's memory is released;
  * a launch whose status word flags non-finite data is swept again one job
    per launch; a job with non-finite data fails (status ENONFINITE in its
    result) and the stream goes on.
Plain mode (the comparison): one job at a time, and one sweep launch per
(reserve ratio, bit-width) candidate.

Every result is independent of the mix: the batched sweep computes each
scene's tables bit-identically to a launch of that scene alone, and the
search is deterministic.
"""
from __future__ import annotations

import os
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import mgs, synth

CHANNELS = 20


def job_device_bytes(n: int, k: np.ndarray, G: int, nb: int) -> int:
    """Device bytes a resident job holds (inputs, kept sets, tables, codes)."""
    T = len(k)
    gm = (int(k.max()) + G - 1) // G
    kmax = int(k.max())
    b = CHANNELS * n * 4 + n * 4                 # attributes, importance
    b += int(k.sum()) * 4                        # kept indices
    b += T * CHANNELS * gm * (nb * 16 + 8)       # err, bits, gmin, gmax
    b += CHANNELS * kmax * 2 + CHANNELS * gm * 9  # codes, final bounds and bit-widths
    b += int(mgs.lib().mgs_prune_select_ws_bytes(n, T))
    return b


class Admission:
    """Admission by device memory: a job is admitted while the resident total
    stays under the cap; a job larger than the cap is admitted only when
    nothing else is resident (so it cannot wait forever)."""

    def __init__(self, cap_bytes: int):
        self.cap = int(cap_bytes)
        self.used = 0
        self.resident = 0

    def try_admit(self, need: int) -> bool:
        if self.resident and self.used + need > self.cap:
            return False
        self.used += need
        self.resident += 1
        return True

    def release(self, need: int):
        self.used -= need
        self.resident -= 1
        assert self.used >= 0 and self.resident >= 0


@dataclass
class JobResult:
    job_id: int
    n: int
    arrival: float          # seconds from the start of the stream
    admitted: float
    swept: float
    solved: float
    done: float
    evals: int
    best_t: int
    best_bits: Optional[np.ndarray]
    codes: Optional[np.ndarray] = None   # u16 [C][k_best] when kept
    status: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Live:
    job: synth.Job
    k: np.ndarray
    need: int
    t_admit: float
    dev: Dict = field(default_factory=dict)
    host: Dict = field(default_factory=dict)
    ev: object = None
    fut: object = None
    res: Optional[dict] = None
    t_swept: float = 0.0
    t_solved: float = 0.0
    status_h: object = None
    batch_n: int = 0       # jobs in the sweep launch that computed its tables


class SceneStore:
    """Pinned host copies of the base scenes the jobs draw from."""

    def __init__(self, num_bases: int = synth.NUM_BASES, n: int = synth.BASE_N):
        import torch
        self.n = n
        self.attr, self.imp = [], []
        for b in range(num_bases):
            a, w = synth.base_scene(b, n)
            self.attr.append(torch.from_numpy(a).pin_memory())
            self.imp.append(torch.from_numpy(w).pin_memory())


class Server:
    """Runs a stream of jobs in batched (continuous batching) or plain mode."""

    def __init__(self, store: SceneStore, G: int = 8192, bits=range(2, 17), mode: str = "batched",
                 mem_cap_bytes: int = 32 << 30, host_workers: int = 4, ilp_threads: int = 0,
                 keep_codes: bool = False, max_batch: int = mgs.MAX_JOBS, warm_up: bool = True,
                 max_inflight: int = 1):
        import torch
        assert mode in ("batched", "plain")
        self.torch = torch
        self.store = store
        self.G = G
        self.bits = [int(b) for b in bits]
        self.nb = len(self.bits)
        self.mode = mode
        self.adm = Admission(mem_cap_bytes if mode == "batched" else 0)  # plain: one job at a time
        self.keep_codes = keep_codes
        self.max_batch = max_batch
        self.max_inflight = max(1, int(max_inflight))
        self.inflight: List = []  # events of the sweep launches on the GPU
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.compute = torch.cuda.Stream()   # default priority
        self.copy = torch.cuda.Stream()
        workers = host_workers if mode == "batched" else 1
        self.pool = ThreadPoolExecutor(max_workers=workers)
        # host threads per ILP search: the cores shared among the pool's workers
        cores = len(os.sched_getaffinity(0))
        self.ilp_threads = ilp_threads if ilp_threads > 0 else max(1, cores // workers)
        self.launches = 0
        self.batch_sizes: List[int] = []
        # workspaces of the batched sweep, one per launch in flight (ring)
        # (descriptors without counts: the size covers any job of up to store.n
        # Gaussians and MAX_RATIOS reserve ratios)
        probe = (mgs.SweepJob * max_batch)()
        for j in range(max_batch):
            probe[j].desc.G = G
            probe[j].desc.N = store.n
            probe[j].desc.T = mgs.MAX_RATIOS
        need = mgs.lib().mgs_quant_sweep_multi_ws_bytes(probe, max_batch)
        self.ws_ring = [mgs.workspace(need, self.dev) for _ in range(8)]
        self.ws_next = 0
        self.plain_ws = mgs.workspace(1 << 22, self.dev)
        if warm_up:
            self._warm_up()

    def _warm_up(self):
        """One small job through every stage before the stream starts: the first
        use of each kernel loads its code object and the first pinned and device
        allocations of each size are slow, which would otherwise land on the
        first jobs' latency.  Nothing of it is kept or counted."""
        n = min(50_000, self.store.n)
        job = synth.Job(-1, 0.0, n, n * 80 // 30, 0, list(synth.job_stream(1)[0].ratios))
        k = synth.keep_counts(job.n, job.ratios)
        live = _Live(job, k, 0, 0.0)
        self._admit(live)
        self._launch_sweep([live])
        live.ev.synchronize()
        live.res = self._solve(live)
        self._launch_codes(live)
        if live.ev is not None:
            live.ev.synchronize()
        live.dev.clear()
        live.host.clear()
        self.launches = 0
        self.batch_sizes.clear()

    # ---- per-job device work -------------------------------------------------
    def _admit(self, live: _Live):
        torch = self.torch
        job, k = live.job, live.k
        n, C, G, nb, T = job.n, CHANNELS, self.G, self.nb, len(k)
        gm = (int(k.max()) + G - 1) // G
        d = live.dev
        with torch.cuda.stream(self.copy):
            d["attr"] = torch.empty((C, n), dtype=torch.float32, device=self.dev)
            d["imp"] = torch.empty(n, dtype=torch.float32, device=self.dev)
            src_a, src_w = self.store.attr[job.base], self.store.imp[job.base]
            for c in range(C):
                d["attr"][c].copy_(src_a[c, :n], non_blocking=True)
            d["imp"].copy_(src_w[:n], non_blocking=True)
            up = torch.cuda.Event()
            up.record(self.copy)
        with torch.cuda.stream(self.compute):
            self.compute.wait_event(up)
            d["kept"] = torch.empty(int(k.sum()), dtype=torch.int32, device=self.dev)
            d["ws_p"] = mgs.workspace(mgs.lib().mgs_prune_select_ws_bytes(n, T), self.dev)
            mgs.prune_select(d["imp"], k, ws=d["ws_p"], out=d["kept"], stream=self.compute, check=False)
            d["out"] = mgs.sweep_tables(T, C, gm, nb, self.dev)
            d["bw"] = torch.empty(C * gm, dtype=torch.uint8, device=self.dev)
            d["codes"] = torch.empty(C * int(k.max()), dtype=torch.int16, device=self.dev)
            d["gmn"] = torch.empty(C * gm, dtype=torch.float32, device=self.dev)
            d["gmx"] = torch.empty(C * gm, dtype=torch.float32, device=self.dev)
            # keep the upload sources alive until the copies are done: they are pinned slices
        h = live.host
        h["err"] = torch.empty((T, C, gm, nb), dtype=torch.float64, pin_memory=True)
        h["bits"] = torch.empty((T, C, gm, nb), dtype=torch.float64, pin_memory=True)
        h["bw"] = torch.empty(C * gm, dtype=torch.uint8, pin_memory=True)

    def _launch_sweep(self, batch: List[_Live]):
        torch = self.torch
        with torch.cuda.stream(self.compute):
            if self.mode == "batched":
                scenes = [{"attr": b.dev["attr"], "imp": b.dev["imp"], "kept": b.dev["kept"], "k": b.k,
                           "out": b.dev["out"]} for b in batch]
                ws = self.ws_ring[self.ws_next]
                self.ws_next = (self.ws_next + 1) % len(self.ws_ring)
                mgs.quant_sweep_multi(scenes, self.G, self.bits, ws=ws, stream=self.compute, check=False)
                self.launches += 1
                status = torch.empty(1, dtype=torch.int32, pin_memory=True)
                status.copy_(ws[:4].view(torch.int32), non_blocking=True)
            else:
                (b,) = batch
                status = self._plain_sweep(b)
            for b in batch:
                b.host["err"].copy_(b.dev["out"]["err"], non_blocking=True)
                b.host["bits"].copy_(b.dev["out"]["bits"], non_blocking=True)
                b.status_h = status
                b.batch_n = len(batch)
            ev = torch.cuda.Event()
            ev.record(self.compute)
        for b in batch:
            b.ev = ev
        self.inflight.append(ev)
        self.batch_sizes.append(len(batch))

    def _plain_sweep(self, b: _Live):
        """One launch per (ratio, bit-width) candidate, each writing its column
        of the job's tables."""
        torch = self.torch
        k, G = b.k, self.G
        offs = np.concatenate([[0], np.cumsum(k)])
        out = b.dev["out"]
        st = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        for t, kt in enumerate(k):
            gm_t = (int(kt) + G - 1) // G
            col = mgs.sweep_tables(1, CHANNELS, gm_t, 1, self.dev)
            kv = b.dev["kept"][int(offs[t]):int(offs[t + 1])]
            for i, bb in enumerate(self.bits):
                mgs.quant_sweep(b.dev["attr"], b.dev["imp"], kv, [int(kt)], G, [bb], ws=self.plain_ws, out=col,
                                stream=self.compute, check=False)
                self.launches += 1
                out["err"][t, :, :gm_t, i].copy_(col["err"][0, :, :, 0])
                out["bits"][t, :, :gm_t, i].copy_(col["bits"][0, :, :, 0])
            out["err"][t, :, gm_t:].fill_(float("nan"))
            out["bits"][t, :, gm_t:].fill_(float("nan"))
        st.copy_(self.plain_ws[:4].view(torch.int32), non_blocking=True)
        return st

    def _solve(self, live: _Live):
        """The job's search; a library error (e.g. the exact ILP's state limit)
        fails this job only, with the code in its result."""
        job = live.job
        try:
            res = mgs.search(job.n, CHANNELS, live.k, self.G, self.bits, live.host["err"].numpy(),
                             live.host["bits"].numpy(), 8 * job.budget_bytes, threads=self.ilp_threads)
            res["code"] = mgs.OK
        except mgs.MgsError as e:
            res = {"best_t": -1, "best_bits": None, "code": e.code}
        return res

    def _launch_codes(self, live: _Live):
        torch = self.torch
        res, k, G, d = live.res, live.k, self.G, live.dev
        t = res["best_t"]
        if t < 0:
            return
        kt = int(k[t])
        ng = (kt + G - 1) // G
        off = int(np.sum(k[:t]))
        live.host["bw"][:CHANNELS * ng].copy_(torch.from_numpy(res["best_bits"].reshape(-1)))
        with torch.cuda.stream(self.compute):
            d["bw"][:CHANNELS * ng].copy_(live.host["bw"][:CHANNELS * ng], non_blocking=True)
            L = mgs.lib()
            kp = d["kept"].data_ptr() + 4 * off
            rc = L.mgs_quantize(d["attr"].data_ptr(), live.job.n, CHANNELS, kp, kt, G, d["bw"].data_ptr(),
                                d["codes"].data_ptr(), d["gmn"].data_ptr(), d["gmx"].data_ptr(),
                                self.compute.cuda_stream)
            if rc:
                raise mgs.MgsError(rc, "mgs_quantize")
            live.host["codes"] = torch.empty(CHANNELS * kt, dtype=torch.int16, pin_memory=True)
            live.host["codes"].copy_(d["codes"][:CHANNELS * kt], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.compute)
        live.ev = ev

    # ---- the loop ------------------------------------------------------------
    def run(self, jobs: List[synth.Job], time_scale: float = 1.0) -> dict:
        """Serve ``jobs`` (arrival times scaled by ``time_scale``); returns the
        per-job results and the stream's latency and throughput figures."""
        torch = self.torch
        G, nb = self.G, self.nb
        pending = deque(sorted(jobs, key=lambda j: j.arrival_s))
        waiting: deque = deque()
        ready: List[_Live] = []
        solo: deque = deque()
        sweeping: List[_Live] = []
        solving: List[_Live] = []
        coding: List[_Live] = []
        results: List[JobResult] = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or waiting or ready or solo or sweeping or solving or coding:
            progressed = False
            tn = now()
            while pending and pending[0].arrival_s * time_scale <= tn:
                waiting.append(pending.popleft())
                progressed = True
            # admission by memory
            while waiting:
                job = waiting[0]
                k = synth.keep_counts(job.n, job.ratios)
                need = job_device_bytes(job.n, k, G, nb)
                if not self.adm.try_admit(need):
                    break
                waiting.popleft()
                live = _Live(job, k, need, now())
                self._admit(live)
                ready.append(live)
                progressed = True
            # jobs of a launch whose status word flagged non-finite data are
            # swept again one per launch, so the flag names the job
            while solo and len(self.inflight) < self.max_inflight:
                one = solo.popleft()
                self._launch_sweep([one])
                sweeping.append(one)
                progressed = True
            # one sweep launch over every ready job (plain: the oldest one),
            # once a launch slot is free: jobs that get ready meanwhile gather
            # for the next launch
            self.inflight = [e for e in self.inflight if not e.query()]
            if ready and len(self.inflight) < self.max_inflight:
                if self.mode == "batched":
                    batch, ready = ready[:self.max_batch], ready[self.max_batch:]
                else:
                    batch, ready = ready[:1], ready[1:]
                self._launch_sweep(batch)
                sweeping.extend(batch)
                progressed = True
            # tables on the host: hand the job to the ILP pool
            for live in [x for x in sweeping if x.ev.query()]:
                sweeping.remove(live)
                live.t_swept = now()
                if int(live.status_h[0]) != 0:
                    if live.batch_n > 1:
                        solo.append(live)  # which job of the launch: sweep it alone
                    else:
                        # this job's data is not finite: it fails, the stream goes on
                        live.res = {"best_t": -1, "best_bits": None, "code": mgs.ENONFINITE}
                        live.t_solved = now()
                        live.ev = None
                        coding.append(live)
                    progressed = True
                    continue
                live.fut = self.pool.submit(self._solve, live)
                solving.append(live)
                progressed = True
            for live in [x for x in solving if x.fut.done()]:
                solving.remove(live)
                live.res = live.fut.result()
                live.t_solved = now()
                self._launch_codes(live)
                coding.append(live)
                progressed = True
            for live in [x for x in coding if x.ev is None or x.ev.query()]:
                coding.remove(live)
                res = live.res
                codes = None
                if self.keep_codes and "codes" in live.host:
                    codes = live.host["codes"].numpy().view(np.uint16).reshape(CHANNELS, -1).copy()
                job = live.job
                results.append(JobResult(job.job_id, job.n, job.arrival_s * time_scale, live.t_admit,
                                         live.t_swept, live.t_solved, now(),
                                         int(live.k.sum()) * CHANNELS * nb, res["best_t"],
                                         None if res["best_bits"] is None else res["best_bits"].copy(), codes,
                                         res["code"]))
                live.dev.clear()
                live.host.clear()
                self.adm.release(live.need)
                progressed = True
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        results.sort(key=lambda r: r.job_id)
        lat = np.array([r.latency for r in results])
        first = min(r.arrival for r in results)
        last = max(r.done for r in results)
        evals = sum(r.evals for r in results)
        return {"results": results,
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "evals_per_s": evals / (last - first), "wall_s": last - first,
                "jobs": len(results), "failed": sum(1 for r in results if r.status != mgs.OK),
                "launches": self.launches,
                "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
                "max_batch": int(max(self.batch_sizes)) if self.batch_sizes else 0}

    def close(self):
        self.pool.shutdown(wait=True)
