"""Seeded synthetic inputs shaped like trained 3DGS scenes.

This module only draws random numbers and lays them out. It holds none of the
quantization, entropy, pruning, assignment or allocation arithmetic, so both
the HIP path and the CPU oracle can take their inputs from it.

Attribute layout (the paper treats the attributes as a 2D matrix split into
channel x block pieces, section "Binary ILP for Q"): structure-of-arrays,
float32 ``attr[C][N]``, channels in this order

    0..2   DC colour (SH degree 0)         ~ Normal(0, 0.5)
    3      opacity logit                   ~ Normal(0, 2)
    4..6   log-scale                       ~ Normal(-4, 1)
    7..10  rotation quaternion             = Normal(0, 1)^4 normalised per Gaussian
    11..19 SH degree 1 (3 coeffs x 3 RGB)  ~ Laplace(0, 0.05)        (C = 20 only)

Importance ~ LogNormal(0, 2) (second argument = sigma of the underlying
normal, NumPy semantics).  Draw order is fixed: importance, DC, opacity,
scale, rotation, SH-1; every draw uses ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional, Sequence

import numpy as np


def scene(n: int, channels: int, seed: int = 0):
    """Return ``(attr f32[C][n] C-contiguous, imp f32[n])``."""
    if channels not in (11, 20):
        raise ValueError("channels must be 11 or 20")
    rng = np.random.default_rng(seed)
    imp = rng.lognormal(0.0, 2.0, n).astype(np.float32)
    attr = np.empty((channels, n), dtype=np.float32)
    attr[0:3] = rng.normal(0.0, 0.5, (3, n))
    attr[3] = rng.normal(0.0, 2.0, n)
    attr[4:7] = rng.normal(-4.0, 1.0, (3, n))
    rot = rng.normal(0.0, 1.0, (4, n))
    rot /= np.sqrt((rot * rot).sum(axis=0, keepdims=True))
    attr[7:11] = rot
    if channels == 20:
        attr[11:20] = rng.laplace(0.0, 0.05, (9, n))
    return attr, imp


def keep_counts(n: int, ratios: Sequence[Fraction]) -> np.ndarray:
    """Number of Gaussians each reserve ratio keeps: floor(n * p / q), exact.

    Reserve ratios are exact rationals so the count never depends on a float
    rounding of tau.
    """
    return np.array([(n * r.numerator) // r.denominator for r in ratios], dtype=np.int64)


def ratios_cfg_small() -> List[Fraction]:
    return [Fraction(p, 10) for p in (3, 5, 7, 9)]


def ratios_uniform(lo: Fraction, hi: Fraction, count: int) -> List[Fraction]:
    """``count`` ratios uniformly spaced over [lo, hi], endpoints included."""
    if count == 1:
        return [lo]
    step = (hi - lo) / (count - 1)
    return [lo + i * step for i in range(count)]


def voxels(n: int, depth: int, seed: int = 0, clusters: int = 8):
    """``n`` distinct occupied voxels of a 2^depth grid, clustered like the
    surfaces of a scene (Gaussian blobs around random centers), as integer
    coordinates i64 [n][3] in random order."""
    rng = np.random.default_rng(seed)
    side = 1 << depth
    assert n <= side ** 3 // 2
    centers = rng.integers(0, side, (clusters, 3))
    out = np.empty((0, 3), np.int64)
    while out.shape[0] < n:
        c = centers[rng.integers(0, clusters, 2 * n)]
        p = np.rint(c + rng.normal(0, side / 8, (2 * n, 3))).astype(np.int64) % side
        out = np.unique(np.concatenate([out, p]), axis=0)
    return out[rng.permutation(out.shape[0])[:n]]


def voxel_codes(coords, depth: int):
    """Morton codes of voxel coordinates (bit 3l + a holds bit l of axis a,
    x = 0, y = 1, z = 2), sorted, with the permutation that sorts them: the
    octree order in which positions reach the attribute transform."""
    coords = np.asarray(coords, dtype=np.uint64)
    code = np.zeros(coords.shape[0], dtype=np.uint64)
    one = np.uint64(1)
    for l in range(depth):
        for a in range(3):
            code |= ((coords[:, a] >> np.uint64(l)) & one) << np.uint64(3 * l + a)
    order = np.argsort(code, kind="stable")
    return code[order], order


def vq_data(n: int, dim: int = 36, k: int = 4096, seed: int = 0):
    """Higher-degree SH vectors ~ Laplace(0, 0.03) and a codebook drawn from them.

    Returns ``(x f32[n][dim], codebook f32[k][dim])``.
    """
    rng = np.random.default_rng(seed)
    x = rng.laplace(0.0, 0.03, (n, dim)).astype(np.float32)
    pick = rng.choice(n, size=k, replace=False)
    return x, np.ascontiguousarray(x[pick])


@dataclass
class SweepWorkload:
    """One sweep workload: scene shape, reserve ratios, group size, bit list."""
    name: str
    n: int
    channels: int
    ratios: List[Fraction]
    group: int
    bits: List[int]
    seed: int = 0
    budget_ratio: Optional[int] = None  # compression ratio of the byte budget

    @property
    def k(self) -> np.ndarray:
        return keep_counts(self.n, self.ratios)

    def make(self):
        return scene(self.n, self.channels, self.seed)

    @property
    def budget_bytes(self) -> Optional[int]:
        if self.budget_ratio is None:
            return None
        return (self.n * self.channels * 4) // self.budget_ratio

    def evals(self) -> int:
        return int(self.k.sum()) * self.channels * len(self.bits)


def workload(name: str) -> SweepWorkload:
    """The sweep workloads used by the tests and the benchmark.

    small  : N=50,000, 11 channels, tau in {0.3,0.5,0.7,0.9}, G=4096, b in 4..8
    medium : N=1,000,000, 20 channels, 16 tau uniformly in [0.2,0.95], G=8192, b in 2..16
    large  : N=5,300,000, 20 channels, 32 tau uniformly in [0.1,0.95], G=16384, b in 1..16,
             byte budget = raw fp32 size / 30
    """
    if name == "small":
        return SweepWorkload("small", 50_000, 11, ratios_cfg_small(), 4096, list(range(4, 9)))
    if name == "medium":
        return SweepWorkload("medium", 1_000_000, 20,
                             ratios_uniform(Fraction(1, 5), Fraction(19, 20), 16),
                             8192, list(range(2, 17)))
    if name == "large":
        return SweepWorkload("large", 5_300_000, 20,
                             ratios_uniform(Fraction(1, 10), Fraction(19, 20), 32),
                             16384, list(range(1, 17)), budget_ratio=30)
    raise KeyError(name)


@dataclass
class Job:
    """One compression request of the serving stream: the first ``n`` Gaussians
    of base scene ``base`` (``scene(BASE_N, 20, seed=1000 + base)``) and a byte
    budget."""
    job_id: int
    arrival_s: float
    n: int
    budget_bytes: int
    base: int
    ratios: List[Fraction] = field(default_factory=list)


BASE_N = 6_000_000   # Gaussians in each base scene of the serving stream
NUM_BASES = 2


def base_scene(base: int, n: int = BASE_N):
    """Base scene ``base`` of the serving stream (its first ``n`` Gaussians)."""
    return scene(n, 20, seed=1000 + base)


def job_stream(num_jobs: int = 64, rate_per_s: float = 2.0, seed: int = 0,
               n_lo: int = 200_000, n_hi: int = BASE_N, num_bases: int = NUM_BASES) -> List[Job]:
    """Poisson arrivals; N log-uniform in [n_lo, n_hi]; budget ratio U(10, 60)
    of the raw FP32 size (20 channels x 4 bytes per Gaussian).

    Each job searches 16 reserve ratios uniformly spaced in [0.2, 0.95].
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, num_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), num_jobs))).astype(np.int64)
    ratio = rng.uniform(10.0, 60.0, num_jobs)
    ratios = ratios_uniform(Fraction(1, 5), Fraction(19, 20), 16)
    jobs = []
    for j in range(num_jobs):
        n = int(ns[j])
        jobs.append(Job(j, float(arrivals[j]), n, int(n * 80 / ratio[j]), j % num_bases, list(ratios)))
    return jobs
