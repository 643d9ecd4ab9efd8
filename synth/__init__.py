"""Seeded synthetic workloads for the exact 1-NN search (random walks and noisy queries).

This module is the only code shared by the test oracle and the GPU path's tests and benchmark.
It produces inputs and nothing else: it holds none of the search method's arithmetic
(no PAA, no iSAX, no lower bound, no distance).

Random-walk generator (Section 4, "Datasets"): the first value is drawn from N(0,1) and every
following value adds a fresh N(0,1) draw to the previous one. Each series is then z-normalised
(mean 0, population standard deviation 1; Section 2.1 relates z-normalised ED to Pearson
correlation) in float64 and stored as float32 (round to nearest).

Streams: ``SeedSequence(seed).spawn(4)`` gives the dataset, query, noise-level and training
streams. The dataset is generated in fixed chunks of ``CHUNK`` series, chunk ``c`` drawing from
``dataset.spawn(n_chunks)[c]``, so the bytes never depend on how many threads ran.

Queries: a source series ``src ~ U{0..N-1}`` plus ``sigma * N(0,1)^n`` noise (computed in
float64 from the float32 source), re-z-normalised, cast to float32. ``sigma`` is either fixed or
drawn per query from ``U[lo, hi]``. ``fresh_walk_queries`` gives the paper's own query workload
(new random walks that are not in the collection).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 1_000_000
STREAM_DATA, STREAM_QUERY, STREAM_SIGMA, STREAM_TRAIN = range(4)


def _streams(seed: int):
    return np.random.SeedSequence(seed).spawn(4)


def _znorm_rows(walk: np.ndarray) -> np.ndarray:
    """z-normalise float64 rows with the population std; returns float32 rows."""
    mu = walk.mean(axis=1, keepdims=True)
    sd = walk.std(axis=1, keepdims=True)  # ddof=0: population std
    sd[sd == 0.0] = 1.0
    return ((walk - mu) / sd).astype(np.float32)


def _walk_chunk(child: np.random.SeedSequence, m: int, n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(child))
    steps = rng.standard_normal((m, n))  # x_0 ~ N(0,1), x_t = x_{t-1} + N(0,1)
    np.cumsum(steps, axis=1, out=steps)
    return _znorm_rows(steps)


def random_walks(n_series: int, length: int, seed: int = 0, out: np.ndarray | None = None,
                 threads: int | None = None) -> np.ndarray:
    """float32 [n_series, length] z-normalised random walks (C order).

    ``out`` may be a preallocated float32 array (e.g. the numpy view of a pinned host tensor).
    """
    if n_series < 0 or length < 1:
        raise ValueError("n_series >= 0 and length >= 1 required")
    if out is None:
        out = np.empty((n_series, length), dtype=np.float32)
    if out.shape != (n_series, length) or out.dtype != np.float32 or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous float32 array of shape (n_series, length)")
    n_chunks = (n_series + CHUNK - 1) // CHUNK
    if n_chunks == 0:
        return out
    children = _streams(seed)[STREAM_DATA].spawn(n_chunks)

    def work(c: int) -> None:
        lo = c * CHUNK
        hi = min(n_series, lo + CHUNK)
        # sub-chunks keep the float64 temporaries small; the draw order inside a chunk is one
        # generator consumed front to back, so splitting the draw preserves the bytes.
        rng = np.random.Generator(np.random.PCG64(children[c]))
        step = 65536
        for a in range(lo, hi, step):
            b = min(hi, a + step)
            w = rng.standard_normal((b - a, length))
            np.cumsum(w, axis=1, out=w)
            out[a:b] = _znorm_rows(w)

    if threads is None:
        threads = min(n_chunks, max(1, min(16, os.cpu_count() or 1)))
    if threads <= 1 or n_chunks == 1:
        for c in range(n_chunks):
            work(c)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, range(n_chunks)))
    return out


def noisy_queries(data: np.ndarray, n_queries: int, seed: int = 0, sigma=0.1):
    """Queries = dataset series + Gaussian noise, re-z-normalised.

    ``sigma`` is a float (fixed noise std) or a ``(lo, hi)`` pair (per-query U[lo, hi]).
    Returns ``(queries float32 [M, n], src int64 [M], sigma float64 [M])``.
    """
    n_series, length = data.shape
    if n_series < 1:
        raise ValueError("empty collection")
    ss = _streams(seed)
    rq = np.random.Generator(np.random.PCG64(ss[STREAM_QUERY]))
    rs = np.random.Generator(np.random.PCG64(ss[STREAM_SIGMA]))
    src = rq.integers(0, n_series, size=n_queries, dtype=np.int64)
    if isinstance(sigma, (tuple, list)):
        sig = rs.uniform(float(sigma[0]), float(sigma[1]), size=n_queries)
    else:
        sig = np.full(n_queries, float(sigma))
    noise = rq.standard_normal((n_queries, length))
    y = data[src].astype(np.float64) + sig[:, None] * noise
    return _znorm_rows(y), src, sig


def fresh_walk_queries(n_queries: int, length: int, seed: int = 0) -> np.ndarray:
    """The paper's own query workload: new random walks drawn from the query stream."""
    child = _streams(seed)[STREAM_QUERY].spawn(1)[0]
    return _walk_chunk(child, n_queries, length)


def training_queries(data: np.ndarray, n_queries: int, seed: int = 0, sigma=(0.05, 0.5)):
    """Noisy queries from the training stream (disjoint from ``noisy_queries``' stream)."""
    n_series, length = data.shape
    tr = _streams(seed)[STREAM_TRAIN]
    rq_ss, rs_ss = tr.spawn(2)
    rq = np.random.Generator(np.random.PCG64(rq_ss))
    rs = np.random.Generator(np.random.PCG64(rs_ss))
    src = rq.integers(0, n_series, size=n_queries, dtype=np.int64)
    if isinstance(sigma, (tuple, list)):
        sig = rs.uniform(float(sigma[0]), float(sigma[1]), size=n_queries)
    else:
        sig = np.full(n_queries, float(sigma))
    noise = rq.standard_normal((n_queries, length))
    y = data[src].astype(np.float64) + sig[:, None] * noise
    return _znorm_rows(y), src, sig


def raw_steps_for_test(n_series: int, length: int, seed: int = 0) -> np.ndarray:
    """The float64 N(0,1) increments of the first chunk, before cumsum and z-normalisation.

    Only for statistical tests of the generator (increment mean/variance).
    """
    m = min(n_series, CHUNK)
    child = _streams(seed)[STREAM_DATA].spawn(max(1, (n_series + CHUNK - 1) // CHUNK))[0]
    rng = np.random.Generator(np.random.PCG64(child))
    return rng.standard_normal((m, length))
