"""Seeded synthetic workloads for SuCo search.

This module only draws random numbers: it holds none of the search method's
arithmetic and is shared by the oracle tests, the GPU tests and the benchmark.
The paper evaluates on public ANN datasets (SIFT, GIST, Deep, SPACEV); none of
their records is used or reproduced here.  Each workload below is a synthetic
stand-in with the shape and value distribution of one of them:

  mixture128  n=10,000   d=128  Gaussian mixture, 100 components, centres N(0,4I)
  sift_like   n=1M       d=128  non-negative integers 0..255, heavy tailed, with
                                a 16-dim latent 1000-cluster structure (SIFT-like)
  gist_like   n=1M       d=960  values in (0,1): sigmoid of a 32-dim latent
                                500-cluster mixture (GIST-like)
  deep_like   n=10M      d=96   unit-norm rows, 10,000 clusters (Deep-like)
  lifted256   n=10M      d=256  16-dim latent 5000-cluster mixture lifted to 256

Seeds: structure (centres, projection matrices) = 1000*c, data = 1000*c+1,
queries = 1000*c+2, training queries = 1000*c+3, batch-size stream = 1000*c+4,
where c is the workload number 1..5.  Rows are drawn in chunks of 2**20 with a
per-chunk child seed so that any row range can be regenerated independently.
"""
from __future__ import annotations

import math

import numpy as np

CHUNK = 1 << 20

WORKLOADS = {
    1: dict(name="mixture128", n=10_000, d=128, n_s=8, sqrt_k=16, nq=100,
            k=10, alpha=0.05, beta=0.005),
    2: dict(name="sift_like", n=1_000_000, d=128, n_s=8, sqrt_k=50, nq=10_000,
            k=10, alpha=0.03, beta=0.005),
    3: dict(name="gist_like", n=1_000_000, d=960, n_s=20, sqrt_k=50, nq=1_000,
            k=10, alpha=0.05, beta=0.005),
    4: dict(name="deep_like", n=10_000_000, d=96, n_s=8, sqrt_k=64, nq=100_000,
            k=10, alpha=0.02, beta=0.002),
    5: dict(name="lifted256", n=10_000_000, d=256, n_s=16, sqrt_k=64, nq=10_000,
            k=10, alpha=0.03, beta=0.003),
}

SEED_STRUCT, SEED_DATA, SEED_QUERY, SEED_TRAIN, SEED_BATCH = 0, 1, 2, 3, 4


def _rng(seed: int, chunk: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, chunk])))


def _norm_cdf(x: np.ndarray) -> np.ndarray:
    from scipy.special import ndtr
    return ndtr(x)


class Workload:
    """A seeded generator for one workload; rows(seed, start, count) is pure."""

    def __init__(self, c: int):
        self.c = c
        self.spec = dict(WORKLOADS[c])
        self.d = self.spec["d"]
        rs = np.random.Generator(np.random.PCG64(1000 * c + SEED_STRUCT))
        if c == 1:
            self.centres = rs.normal(0.0, 2.0, size=(100, 128))
        elif c == 2:
            self.centres = rs.normal(0.0, 1.0, size=(1000, 16))
            self.W = rs.normal(0.0, 1.0 / 4.0, size=(128, 16))
            self.sd = np.sqrt((self.W ** 2).sum(axis=1) * 1.25)
        elif c == 3:
            self.centres = rs.normal(0.0, 1.0, size=(500, 32))
            self.A = rs.normal(0.0, 1.0 / math.sqrt(32.0), size=(960, 32))
        elif c == 4:
            self.centres = rs.normal(0.0, 1.0, size=(10_000, 96))
        elif c == 5:
            self.centres = rs.normal(0.0, 1.0, size=(5000, 16))
            self.M = rs.normal(0.0, 0.25, size=(256, 16))
        else:
            raise ValueError(f"unknown workload {c}")

    def _draw(self, rng: np.random.Generator, m: int) -> np.ndarray:
        c = self.c
        if c == 1:
            lab = rng.integers(0, 100, size=m)
            x = self.centres[lab] + rng.normal(0.0, 1.0, size=(m, 128))
        elif c == 2:
            lab = rng.integers(0, 1000, size=m)
            z = self.centres[lab] + rng.normal(0.0, 0.5, size=(m, 16))
            y = z @ self.W.T
            u = _norm_cdf(y / self.sd)
            u = np.minimum(u, 1.0 - 1e-16)
            x = np.rint(np.minimum(255.0, -20.0 * np.log1p(-u)))
        elif c == 3:
            lab = rng.integers(0, 500, size=m)
            z = self.centres[lab] + rng.normal(0.0, 0.5, size=(m, 32))
            x = 1.0 / (1.0 + np.exp(-(z @ self.A.T + 0.1 * rng.normal(size=(m, 960)))))
        elif c == 4:
            lab = rng.integers(0, 10_000, size=m)
            v = self.centres[lab] + 0.3 * rng.normal(size=(m, 96))
            x = v / np.linalg.norm(v, axis=1, keepdims=True)
        else:
            lab = rng.integers(0, 5000, size=m)
            z = self.centres[lab] + rng.normal(0.0, 0.5, size=(m, 16))
            x = z @ self.M.T + 0.05 * rng.normal(size=(m, 256))
        return np.ascontiguousarray(x, dtype=np.float32)

    def rows(self, seed_kind: int, count: int, start: int = 0) -> np.ndarray:
        """Rows [start, start+count) of the stream with the given seed kind."""
        seed = 1000 * self.c + seed_kind
        out = np.empty((count, self.d), dtype=np.float32)
        pos = start
        while pos < start + count:
            ch = pos // CHUNK
            c0 = ch * CHUNK
            take_hi = min(start + count, c0 + CHUNK)
            block = self._draw(_rng(seed, ch), min(CHUNK, take_hi - c0))
            out[pos - start:take_hi - start] = block[pos - c0:take_hi - c0]
            pos = take_hi
        return out

    def data(self, n: int | None = None) -> np.ndarray:
        return self.rows(SEED_DATA, self.spec["n"] if n is None else n)

    def queries(self, nq: int | None = None) -> np.ndarray:
        return self.rows(SEED_QUERY, self.spec["nq"] if nq is None else nq)

    def train_queries(self, m: int, start: int = 0) -> np.ndarray:
        return self.rows(SEED_TRAIN, m, start)

    def batch_sizes(self, total: int, max_batch: int = 4096) -> list[int]:
        """Uneven batch sizes uniform in 1..max_batch summing to total."""
        rng = np.random.Generator(np.random.PCG64(1000 * self.c + SEED_BATCH))
        out, left = [], total
        while left > 0:
            b = int(rng.integers(1, max_batch + 1))
            b = min(b, left)
            out.append(b)
            left -= b
        return out


def tiny(n: int, d: int, seed: int, kind: str = "gauss", levels: int = 0) -> np.ndarray:
    """Small random matrices for property tests.

    kind="gauss": N(0,1); kind="int": integers in [0, levels) (forces ties);
    kind="clustered": a few tight clusters.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "gauss":
        x = rng.normal(size=(n, d))
    elif kind == "int":
        x = rng.integers(0, max(levels, 2), size=(n, d)).astype(np.float64)
    elif kind == "clustered":
        cen = rng.normal(0.0, 3.0, size=(max(2, n // 20), d))
        x = cen[rng.integers(0, cen.shape[0], size=n)] + 0.3 * rng.normal(size=(n, d))
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(x, dtype=np.float32)
