"""Chunked, seeded generators for the synthetic workloads.

Every random stream is a numpy ``SeedSequence(seed, spawn_key=...)`` of its
own, so any chunk of 2**20 database rows (and any prefix of it) can be drawn
alone and always yields the same values:

  (0, c)      dataset-level parameters (mixture centres, per-dim scales)
  (1, i, c)   database chunk i, component c
  (2, 0, c)   queries, component c
  (3, 0, c)   serving request stream (arrival gaps, nprobe, k)

Rows are float32, row-major.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .workloads import Workload

CHUNK = 1 << 20


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed, spawn_key=key))


def _params(w: Workload):
    """Dataset-level parameters shared by every chunk and by the queries."""
    if w.kind == "mixture":
        return _rng(w.seed, 0, 0).standard_normal((w.centres, w.d))
    if w.kind == "unit_mixture":
        c = _rng(w.seed, 0, 0).standard_normal((w.centres, w.d))
        return c / np.linalg.norm(c, axis=1, keepdims=True)
    if w.kind == "gamma_int":
        # per-dimension scale theta_d = 10 + 30 U(0,1)
        return 10.0 + 30.0 * _rng(w.seed, 0, 1).random(w.d)
    if w.kind == "blocks_abs":
        return None
    raise ValueError(f"unknown workload kind {w.kind!r}")


def _rows(w: Workload, params, stream: tuple, rows: int) -> np.ndarray:
    """Draw ``rows`` rows of the recipe from the streams ``stream + (c,)``."""
    s = w.seed
    if w.kind in ("mixture", "unit_mixture"):
        lab = _rng(s, *stream, 0).integers(0, params.shape[0], size=rows)
        noise = _rng(s, *stream, 1).standard_normal((rows, w.d))
        x = params[lab] + w.sigma * noise
        if w.kind == "unit_mixture":
            x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x.astype(np.float32)
    if w.kind == "gamma_int":
        g = np.empty((rows, w.d), np.float32)
        _rng(s, *stream, 0).standard_gamma(1.5, out=g, dtype=np.float32)
        g *= params.astype(np.float32)
        np.rint(g, out=g)
        np.clip(g, 0.0, 255.0, out=g)
        return g
    if w.kind == "blocks_abs":
        nb = 64
        assert w.d % nb == 0, "blocks_abs needs D divisible by 64"
        per = w.d // nb
        gblk = _rng(s, *stream, 0).standard_normal((rows, nb), dtype=np.float32)
        eps = _rng(s, *stream, 1).standard_normal((rows, w.d), dtype=np.float32)
        x = 0.8 * np.repeat(gblk, per, axis=1) + 0.6 * eps
        return np.abs(x, out=x)
    raise ValueError(w.kind)


def database(w: Workload, start: int = 0, stop: int | None = None,
             out: np.ndarray | None = None, threads: int | None = None) -> np.ndarray:
    """Rows [start, stop) of the database of ``w`` as float32 (stop-start) x d."""
    stop = w.n if stop is None else stop
    if not 0 <= start <= stop <= w.n:
        raise ValueError("row range out of bounds")
    n = stop - start
    if out is None:
        out = np.empty((n, w.d), np.float32)
    assert out.shape == (n, w.d) and out.dtype == np.float32
    params = _params(w)
    first, last = start // CHUNK, (stop - 1) // CHUNK if n else -1
    jobs = []
    for ci in range(first, last + 1):
        c0 = ci * CHUNK
        lo, hi = max(start, c0), min(stop, c0 + CHUNK)
        jobs.append((ci, c0, lo, hi))

    def run(job):
        ci, c0, lo, hi = job
        block = _rows(w, params, (1, ci), hi - c0)  # prefix of chunk ci
        out[lo - start:hi - start] = block[lo - c0:hi - c0]

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if len(jobs) <= 1 or threads <= 1:
        for j in jobs:
            run(j)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, jobs))
    return out


def queries(w: Workload, nq: int | None = None) -> np.ndarray:
    """``nq`` queries drawn from the same recipe as the database (own stream)."""
    nq = w.nq if nq is None else nq
    return _rows(w, _params(w), (2, 0), nq)


def arrivals(rate_qps: float, count: int, seed: int = 0):
    """Open-loop Poisson request stream for the serving workload.

    Returns (arrival times in seconds, nprobe per request, k per request):
    exponential gaps at ``rate_qps``, nprobe uniform over {8, 16, ..., 256},
    k uniform over {10, 100}.
    """
    gaps = _rng(seed, 3, 0, 0).exponential(1.0 / rate_qps, size=count)
    t = np.cumsum(gaps)
    nprobe = 8 * _rng(seed, 3, 0, 1).integers(1, 33, size=count)
    k = np.where(_rng(seed, 3, 0, 2).integers(0, 2, size=count) == 0, 10, 100)
    return t, nprobe.astype(np.int32), k.astype(np.int32)
