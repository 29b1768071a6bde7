"""Seeded synthetic workloads for the dynamic graph index.

This module only draws random numbers. It holds none of the index's
arithmetic (no distances, no pruning, no search), so both the GPU path and the
CPU oracle can consume what it produces without sharing method code.

The paper evaluates on public vector datasets (Section 5.2, dataset table) that
are not available here. The mixtures below stand in for them: clustered
Gaussian mixtures with the dimensions, dtypes and churn rates of the five
workloads this project measures.

Streams: every workload takes one integer seed and spawns independent child
streams with ``numpy.random.SeedSequence``, one per purpose, so that e.g. the
number of queries drawn never perturbs the vectors inserted.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional

import numpy as np

METRIC_L2_U8 = 0
METRIC_IP_F32 = 1

# Child-stream order (fixed; appending new purposes at the end keeps old ones).
_STREAMS = ("centers", "base", "queries", "deletes", "inserts", "rounds", "arrivals")


def _rngs(seed: int) -> dict:
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(len(_STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k)) for name, k in zip(_STREAMS, kids)}


@dataclasses.dataclass
class Mixture:
    """A clustered Gaussian mixture.

    u8 form: centers uniform in [lo, hi]^dim; a point is its center plus
    N(0, sigma^2) noise per dimension, rounded half-to-even and clamped to
    [0, 255].

    float form: centers N(0, I) normalised to unit length; a point is its
    center plus N(0, sigma^2 I) noise, renormalised (float64), then cast to
    float32.
    """

    dim: int
    n_clusters: int
    sigma: float
    metric: int
    lo: float = 20.0
    hi: float = 235.0

    def centers(self, rng: np.random.Generator) -> np.ndarray:
        if self.metric == METRIC_L2_U8:
            return rng.uniform(self.lo, self.hi, size=(self.n_clusters, self.dim))
        c = rng.standard_normal(size=(self.n_clusters, self.dim))
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        return c

    def draw(self, rng: np.random.Generator, centers: np.ndarray, n: int, with_labels: bool = False,
             allowed: Optional[np.ndarray] = None):
        """n points; with_labels also returns each point's cluster. With
        `allowed` (cluster ids) the labels are drawn uniformly from those
        clusters only; without it the draws are exactly those of the plain
        call (the same stream consumption)."""
        if allowed is None:
            labels = rng.integers(0, self.n_clusters, size=n)
        else:
            allowed = np.asarray(allowed)
            labels = allowed[rng.integers(0, allowed.size, size=n)]
        out = np.empty((n, self.dim), dtype=np.uint8 if self.metric == METRIC_L2_U8 else np.float32)
        chunk = 1 << 16
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            noise = rng.standard_normal(size=(e - s, self.dim)) * self.sigma
            pts = centers[labels[s:e]] + noise
            if self.metric == METRIC_L2_U8:
                out[s:e] = np.clip(np.rint(pts), 0, 255).astype(np.uint8)
            else:
                pts /= np.linalg.norm(pts, axis=1, keepdims=True)
                out[s:e] = pts.astype(np.float32)
        return (out, labels) if with_labels else out


@dataclasses.dataclass
class Workload:
    """One of the five measured workloads (sizes as the project measures them)."""

    name: str
    mixture: Mixture
    n_base: int
    R: int
    L_build: int
    alpha_num: int
    alpha_den: int
    churn_rounds: int
    churn_frac: float
    n_queries: int
    k: int
    search_L: tuple
    seed: int = 0
    build_batch: int = 1000      # the first (bootstrap) batch
    build_batch_max: int = 10000  # later batches double up to this size

    @property
    def metric(self) -> int:
        return self.mixture.metric

    @property
    def dim(self) -> int:
        return self.mixture.dim

    def churn_count(self) -> int:
        return int(round(self.churn_frac * self.n_base))

    def id_capacity(self) -> int:
        return self.n_base + self.churn_rounds * self.churn_count() + 16

    def build_batches(self) -> List[int]:
        """Sizes of the build batches: a bootstrap batch, then doubling up to a cap."""
        sizes, done = [], 0
        b = min(self.build_batch, self.n_base)
        while done < self.n_base:
            b = min(b, self.n_base - done)
            sizes.append(b)
            done += b
            b = min(self.build_batch_max, max(b, done))
        return sizes


def tiny_u8(n_base: int = 10_000, rounds: int = 5, n_queries: int = 1000, seed: int = 0) -> Workload:
    """128-d uint8, 32-cluster mixture, R=32, L=64, alpha=1.2, 1% churn."""
    return Workload("tiny_u8_10k", Mixture(128, 32, 18.0, METRIC_L2_U8), n_base, 32, 64, 6, 5,
                    rounds, 0.01, n_queries, 10, (64,), seed, 1000, 1000)


def scale_u8(n_base: int = 1_000_000, rounds: int = 20, n_queries: int = 10_000, seed: int = 0) -> Workload:
    """128-d uint8, 1,024-cluster mixture, R=32, L=64, alpha=1.2, 1% churn, L in {32,64,128}."""
    return Workload("scale_u8_1m", Mixture(128, 1024, 18.0, METRIC_L2_U8), n_base, 32, 64, 6, 5,
                    rounds, 0.01, n_queries, 10, (32, 64, 128), seed, 1000, 10000)


def precision_f32(n_base: int = 1_000_000, rounds: int = 20, n_queries: int = 10_000, seed: int = 0) -> Workload:
    """768-d unit-norm float32, 2,000 centers, noise 0.35, inner product, R=48, L=96."""
    return Workload("precision_f32_768d_1m", Mixture(768, 2000, 0.35, METRIC_IP_F32), n_base, 48, 96, 6, 5,
                    rounds, 0.01, n_queries, 10, (96,), seed, 1000, 10000)


def serving_u8(n_base: int = 10_000_000, seed: int = 0) -> Workload:
    """128-d uint8 from a 4,096-cluster mixture (sigma 18) at 10M vectors,
    served as a request stream (see Stream.trace and Stream.kinds)."""
    return Workload("serving_u8_10m", Mixture(128, 4096, 18.0, METRIC_L2_U8), n_base, 32, 64, 6, 5,
                    0, 0.0, 0, 10, (64,), seed, 1000, 100_000)


def batching_f32(n_base: int = 4_000_000, rounds: int = 50, seed: int = 0) -> Workload:
    """96-d unit-norm float32, 4,096 centers, noise 0.3, inner product, R=32,
    L=64; rounds of uneven size (see Stream.round_params)."""
    return Workload("batching_f32_96d_4m", Mixture(96, 4096, 0.3, METRIC_IP_F32), n_base, 32, 64, 6, 5,
                    rounds, 0.05, 0, 10, (64,), seed, 1000, 200_000)


class Stream:
    """Draws the vectors of one workload in a fixed order from independent streams."""

    def __init__(self, wl: Workload):
        self.wl = wl
        self.rng = _rngs(wl.seed)
        self.centers = wl.mixture.centers(self.rng["centers"])

    def base(self, n: int) -> np.ndarray:
        return self.wl.mixture.draw(self.rng["base"], self.centers, n)

    def base_labeled(self, n: int):
        """base(n) and the cluster of each point (the same draws as base(n))."""
        return self.wl.mixture.draw(self.rng["base"], self.centers, n, with_labels=True)

    def inserts(self, n: int, clusters: Optional[np.ndarray] = None) -> np.ndarray:
        return self.wl.mixture.draw(self.rng["inserts"], self.centers, n, allowed=clusters)

    def queries(self, n: int, clusters: Optional[np.ndarray] = None) -> np.ndarray:
        return self.wl.mixture.draw(self.rng["queries"], self.centers, n, allowed=clusters)

    def deletes(self, live_ids: np.ndarray, n: int) -> np.ndarray:
        """n distinct ids drawn uniformly without replacement from live_ids, sorted."""
        n = min(n, live_ids.size)
        pick = self.rng["deletes"].choice(live_ids.size, size=n, replace=False)
        return np.sort(live_ids[pick]).astype(np.uint32)

    def uniform_ints(self, lo: int, hi: int, n: int) -> np.ndarray:
        return self.rng["rounds"].integers(lo, hi, size=n)

    def trace(self, rate: float, seconds: float, t0: float = 0.0, p_insert: float = 0.05,
              p_delete: float = 0.05) -> dict:
        """Poisson arrivals at `rate` per second for `seconds`: arrival times,
        and for each request its kind (0 search, 1 insert, 2 delete)."""
        r = self.rng["arrivals"]
        n_est = int(rate * seconds * 1.2) + 16
        t = t0 + np.cumsum(r.exponential(1.0 / rate, size=n_est))
        t = t[t < t0 + seconds]
        u = r.random(t.size)
        kind = np.where(u < p_insert, 1, np.where(u < p_insert + p_delete, 2, 0)).astype(np.uint32)
        return {"t": t, "kind": kind}

    def kinds(self, n: int, p_insert: float = 0.05, p_delete: float = 0.05) -> np.ndarray:
        """Request kinds only (0 search, 1 insert, 2 delete), for streams whose
        arrival times do not matter (saturated serving)."""
        u = self.rng["arrivals"].random(n)
        return np.where(u < p_insert, 1, np.where(u < p_insert + p_delete, 2, 0)).astype(np.uint32)

    def round_params(self, live: int) -> dict:
        """One uneven round: churn fraction drawn from {0.1%, 1%, 5%} of the
        live count (that many deletes and as many inserts), a log-uniform
        query count in [1, 65536], and k drawn from {10, 100}."""
        r = self.rng["rounds"]
        frac = (0.001, 0.01, 0.05)[int(r.integers(0, 3))]
        n = int(round(frac * live))
        nq = log_uniform_batch(r, 1, 65536)
        k = (10, 100)[int(r.integers(0, 2))]
        return {"churn_frac": frac, "n_del": n, "n_ins": n, "n_q": nq, "k": k}


def churn_schedule(wl: Workload) -> Iterator[int]:
    for _ in range(wl.churn_rounds):
        yield wl.churn_count()


def log_uniform_batch(rng: np.random.Generator, lo: int = 1, hi: int = 65536) -> int:
    return int(min(hi, max(lo, math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))))
