"""Autotuner for the factorization's tile shape (panel width).

The panel width is the column count of the panels the factorization and
the solves process per step: it sets the K of the panel kernels, the number
of sequential panel rounds of large supernodes and the tile shapes of the
update kernels' K loop.  The tuner times graph replays of the whole
factorization for each candidate on the device at hand and keeps the
fastest; results are cached per device name and size class (log2 buckets of
n and of the algorithmic flops).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import BatchCholesky, SparseCholesky

CANDIDATES = (16, 32, 48, 64)
_mem_cache: dict = {}


def _cache_path():
    return os.environ.get("SPCHOL_TUNE_CACHE")


def _load():
    p = _cache_path()
    if p and os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return {}


def _store(d):
    p = _cache_path()
    if p:
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)


def size_class(n: int, flops: float) -> str:
    return f"n{int(math.log2(max(n, 1)))}_f{int(math.log2(max(flops, 1.0)))}"


def _device_key():
    import torch
    return torch.cuda.get_device_name(0).replace(" ", "_")


def _time_graph(make_sym, vals, reps):
    import torch
    S = make_sym()
    F = S.factor(vals)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        G = F.capture(vals, stream=stream)
        G.replay(stream)  # warm
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.replay(stream)
        stream.synchronize()
        dt = (time.perf_counter() - t0) / reps
    ok = F.status(stream) == 0
    G.close()
    return dt if ok else math.inf, S


def tune(make_sym_for_width, vals, n: int, flops: float, reps: int = 5, candidates=CANDIDATES,
         use_cache: bool = True):
    """Pick the panel width.  make_sym_for_width(nb) -> SparseCholesky /
    BatchCholesky analysed with that width; vals: the float64 CUDA values.
    Returns (best_width, {width: seconds})."""
    key = f"{_device_key()}/{size_class(n, flops)}"
    if use_cache:
        d = _mem_cache or _load()
        if key in d:
            return int(d[key]["best"]), d[key]["times"]
    times = {}
    for nb in candidates:
        dt, _ = _time_graph(lambda: make_sym_for_width(nb), vals, reps)
        times[int(nb)] = dt
    best = min(times, key=times.get)
    d = _load()
    d[key] = {"best": best, "times": {str(k): v for k, v in times.items()}}
    _mem_cache.update(d)
    _store(d)
    return best, times


def tune_batch(mats, vals, reps: int = 5, amalg_max_zeros: int = 0, candidates=CANDIDATES, use_cache=True):
    """Tune a batch given as (n, colptr, rowind, perm) tuples."""
    probe = BatchCholesky(mats, amalg_max_zeros=amalg_max_zeros)
    inf = probe.info()
    return tune(lambda nb: BatchCholesky(mats, amalg_max_zeros=amalg_max_zeros, panel_width=nb), vals,
                inf["n"], inf["flops_alg"], reps, candidates, use_cache)


def tune_single(n, colptr, rowind, perm, vals, reps: int = 5, amalg_max_zeros: int = 0, candidates=CANDIDATES,
                use_cache=True):
    probe = SparseCholesky(n, colptr, rowind, perm, amalg_max_zeros=amalg_max_zeros)
    inf = probe.info()
    return tune(lambda nb: SparseCholesky(n, colptr, rowind, perm, amalg_max_zeros=amalg_max_zeros, panel_width=nb),
                vals, inf["n"], inf["flops_alg"], reps, candidates, use_cache)
