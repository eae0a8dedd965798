"""Seeded synthetic workloads for the RBC / brute-force k-NN path.

This module holds input generators only -- no distance, ranking or search
arithmetic -- so that the GPU library and the CPU oracle can both be fed the
identical float32 arrays without sharing any of the method's code.

Five workloads stand in for the paper's datasets (which are not available):

  ``iid16``      n=10,000 d=16, X and Q i.i.d. N(0,1), n_r=100
  ``sub8``       n=1,000,000 d=64: an 8-dim linear subspace (random orthonormal
                 embedding, N(0,1) coordinates) plus N(0, 0.01^2) noise,
                 m=10,000, n_r=1,000 (the headline workload)
  ``zipf128``    n=2,000,000 d=128: 2,000 Gaussian clusters (centres U[0,255],
                 sigma 8) with Zipf(1.1) sizes, clamped to [0,255] and rounded to
                 integers, m=20,000, n_r=1,414, s=2,000 (one-shot)
  ``sub16``      n=4,000,000 d=128: 16-dim subspace + N(0, 0.02^2) noise,
                 m=50,000, n_r=2,000
  ``sub12``      n=2,000,000 d=96: 12-dim subspace + N(0, 0.01^2) noise,
                 n_r=1,414, a 200,000-query pool for the serving trace

Seeds: workload number N in 1..5 uses default_rng(10N+1) for the database,
10N+2 for queries, 10N+3 for representatives and 10N+4 for arrivals.  Values
are drawn in float64 and stored as float32.  Rows are generated in fixed
chunks of ``CHUNK`` rows, so a workload is reproducible at any size and a
smaller ``n`` gives a prefix-consistent sample of the same distribution.
"""
from __future__ import annotations

import dataclasses

import numpy as np

CHUNK = 65536


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    number: int
    n: int
    d: int
    m: int
    n_r: int
    s: int = 0


WORKLOADS = {
    "iid16": Workload("iid16", 1, 10_000, 16, 1_000, 100),
    "sub8": Workload("sub8", 2, 1_000_000, 64, 10_000, 1_000),
    "zipf128": Workload("zipf128", 3, 2_000_000, 128, 20_000, 1_414, 2_000),
    "sub16": Workload("sub16", 4, 4_000_000, 128, 50_000, 2_000),
    "sub12": Workload("sub12", 5, 2_000_000, 96, 200_000, 1_414),
}

# subspace generators: (intrinsic dim, noise sigma)
_SUBSPACE = {"sub8": (8, 0.01), "sub16": (16, 0.02), "sub12": (12, 0.01)}


def _seeds(w: Workload):
    b = 10 * w.number
    return b + 1, b + 2, b + 3, b + 4


def _chunks(rows):
    """Full CHUNK-row blocks covering ``rows`` (the last one is truncated after
    drawing, so the random stream does not depend on ``rows``)."""
    for s in range(0, rows, CHUNK):
        yield s, min(rows, s + CHUNK)


def _iid(rng, rows, d):
    out = np.empty((rows, d), np.float32)
    for s, e in _chunks(rows):
        out[s:e] = rng.standard_normal((CHUNK, d))[: e - s]
    return out


def _basis(rng, d, k):
    """Random orthonormal d x k embedding (Q factor of a Gaussian matrix, with
    the signs fixed so that R has a positive diagonal)."""
    g = rng.standard_normal((d, k))
    u, r = np.linalg.qr(g)
    return u * np.sign(np.diag(r))[None, :]


def _subspace(rng, rows, basis, sigma):
    d, k = basis.shape
    out = np.empty((rows, d), np.float32)
    for s, e in _chunks(rows):
        z = rng.standard_normal((CHUNK, k))[: e - s]
        eps = rng.standard_normal((CHUNK, d))[: e - s]
        out[s:e] = z @ basis.T + sigma * eps
    return out


def _zipf_setup(rng, d, n_clusters=2000, a=1.1):
    centres = rng.uniform(0.0, 255.0, size=(n_clusters, d))
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-a)
    return centres, w / w.sum()


def _zipf_rows(rng, rows, centres, p, sigma=8.0):
    d = centres.shape[1]
    out = np.empty((rows, d), np.float32)
    for s, e in _chunks(rows):
        lab = rng.choice(centres.shape[0], size=CHUNK, p=p)[: e - s]
        x = centres[lab] + sigma * rng.standard_normal((CHUNK, d))[: e - s]
        out[s:e] = np.rint(np.clip(x, 0.0, 255.0))
    return out


def database(name: str, n: int | None = None) -> np.ndarray:
    """The database X (n x d float32) of a workload."""
    w = WORKLOADS[name]
    n = w.n if n is None else n
    sd, _, _, _ = _seeds(w)
    rng = np.random.default_rng(sd)
    if name == "iid16":
        return _iid(rng, n, w.d)
    if name == "zipf128":
        centres, p = _zipf_setup(rng, w.d)
        return _zipf_rows(rng, n, centres, p)
    k, sigma = _SUBSPACE[name]
    basis = _basis(rng, w.d, k)
    return _subspace(rng, n, basis, sigma)


def queries(name: str, m: int | None = None) -> np.ndarray:
    """Queries (m x d float32) from the same distribution as the database
    (same embedding or cluster centres, independent draws)."""
    w = WORKLOADS[name]
    m = w.m if m is None else m
    sd, sq, _, _ = _seeds(w)
    rng = np.random.default_rng(sq)
    if name == "iid16":
        return _iid(rng, m, w.d)
    if name == "zipf128":
        centres, p = _zipf_setup(np.random.default_rng(sd), w.d)
        return _zipf_rows(rng, m, centres, p)
    k, sigma = _SUBSPACE[name]
    basis = _basis(np.random.default_rng(sd), w.d, k)
    return _subspace(rng, m, basis, sigma)


def representatives(name: str, n: int | None = None, n_r: int | None = None) -> np.ndarray:
    """n_r distinct database ids drawn uniformly without replacement, sorted."""
    w = WORKLOADS[name]
    n = w.n if n is None else n
    n_r = w.n_r if n_r is None else n_r
    _, _, sr, _ = _seeds(w)
    rng = np.random.default_rng(sr)
    return np.sort(rng.choice(n, size=n_r, replace=False)).astype(np.int64)


def random_reps(n: int, n_r: int, seed: int) -> np.ndarray:
    """Representative ids for ad-hoc sizes (tests)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=n_r, replace=False)).astype(np.int64)


def arrival_trace(name: str, rate: float, n_requests: int, pool: int,
                  mu: float = 4.0, sigma: float = 1.5, max_size: int = 4096):
    """Open-loop serving trace: Poisson arrival times (seconds) at ``rate``
    requests/s, request sizes round(exp(N(mu, sigma^2))) clipped to
    [1, max_size], k uniform over {1, 10}, and each request's query offset in
    the query pool."""
    w = WORKLOADS[name]
    _, _, _, sa = _seeds(w)
    rng = np.random.default_rng(sa + int(rate * 1000) * 7919)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    sizes = np.clip(np.rint(np.exp(rng.normal(mu, sigma, size=n_requests))), 1, max_size)
    sizes = sizes.astype(np.int64)
    ks = np.where(rng.random(n_requests) < 0.5, 1, 10).astype(np.int64)
    offs = rng.integers(0, max(1, pool - max_size), size=n_requests).astype(np.int64)
    return t, sizes, ks, offs
