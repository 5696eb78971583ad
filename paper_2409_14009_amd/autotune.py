"""Autotuner for the shapes the factorization works in.

Three knobs set the shapes of the dense blocks every kernel processes:
  * the supernode granularity (amalgamation): how wide the dense diagonal
    blocks and panels are and how many levels the schedule has -- the
    per-column zero cap z or the paper's greedy merging with a storage cap
    (Sec. IV-A);
  * the panel width: the column count of the panels the factorization and
    the solves process per step (the K of the panel kernels, the number of
    sequential panel rounds of a wide supernode);
  * the update method: 64 x 64 update tiles scattered through per-row
    relative indices (RL), or tiles cut along blocks of consecutive rows
    with one relative index per block (RLB, Sec. II-B, with partition
    refinement).
The tuner times graph replays of the whole factorization (and, when given a
right-hand side block, the solve in the same graph) on the device at hand,
axis by axis (granularity, then panel width, then update method, each time
keeping the best so far), and caches the winner per device, size class
(log2 buckets of n and of the algorithmic flops), update precision and the
search space.  `tune` / `tune_batch` / `tune_single` tune the panel width
alone.
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


# --- the whole analysis configuration ----------------------------------------

AMALG_CHOICES = (("zeros", 8), ("zeros", 32), ("greedy", 25), ("greedy", 50), ("greedy", 100))
WIDTH_CHOICES = (32, 64)
UPDATE_CHOICES = ("rl", "rlb")


def config_kwargs(cfg: dict) -> dict:
    """Keyword arguments of SparseCholesky / BatchCholesky for a config."""
    kind, val = cfg["amalg"]
    kw = dict(panel_width=int(cfg["panel_width"]))
    if kind == "zeros":
        kw.update(amalg_rule=0, amalg_max_zeros=int(val))
    else:
        kw.update(amalg_rule=1, amalg_cap_percent=int(val))
    if cfg["update"] == "rlb":
        kw.update(update_method="rlb", partition_refinement=True)
    return kw


def _time_config(make_sym, cfg, vals, B, precision, reps):
    import torch
    S = make_sym(config_kwargs(cfg))
    F = S.factor(vals, precision=precision)
    stream = torch.cuda.Stream()
    X = None if B is None else torch.empty_like(B)
    with torch.cuda.stream(stream):
        G = F.capture(vals, X, stream=stream)
        if X is not None:
            X.copy_(B)
        G.replay(stream)  # warm
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.replay(stream)
        stream.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ok = F.status(stream) == 0
    G.close()
    del F, S
    return dt if ok else math.inf


def tune_config(make_sym, vals, n: int, flops: float, B=None, precision: str = "f64", reps: int = 5,
                use_cache: bool = True, amalg=AMALG_CHOICES, widths=WIDTH_CHOICES, updates=UPDATE_CHOICES):
    """make_sym(kwargs) -> SparseCholesky / BatchCholesky analysed with those
    options; vals: float64 CUDA values; B: optional (nrhs, n) block solved in
    the same graph.  Returns (best config dict, {config label: seconds})."""
    space = json.dumps([list(map(list, amalg)), list(widths), list(updates)], sort_keys=True)
    nrhs = 0 if B is None else int(B.shape[0])
    import hashlib
    sig = hashlib.sha1(space.encode()).hexdigest()[:10]
    key = f"{_device_key()}/{size_class(n, flops)}/{precision}/rhs{nrhs}/{sig}"
    if use_cache:
        d = _mem_cache or _load()
        if key in d and "config" in d[key]:
            c = d[key]["config"]
            return dict(amalg=tuple(c["amalg"]), panel_width=c["panel_width"], update=c["update"]), d[key]["times"]
    label = lambda c: f"{c['amalg'][0]}{c['amalg'][1]}/nb{c['panel_width']}/{c['update']}"
    times = {}

    def measure(c):
        lb = label(c)
        if lb not in times:
            times[lb] = _time_config(make_sym, c, vals, B, precision, reps)
        return times[lb]

    best = dict(amalg=tuple(amalg[0]), panel_width=int(widths[-1]), update=updates[0])
    for axis, choices in (("amalg", [tuple(a) for a in amalg]), ("panel_width", list(widths)),
                          ("update", list(updates))):
        cands = [dict(best, **{axis: ch}) for ch in choices]
        best = min(cands, key=measure)
    d = _load()
    d[key] = {"config": dict(amalg=list(best["amalg"]), panel_width=best["panel_width"], update=best["update"]),
              "times": times}
    _mem_cache.update(d)
    _store(d)
    return best, times


def tune_batch_config(mats, vals, B=None, precision="f64", reps: int = 5, use_cache=True, **space):
    """tune_config for a batch of (n, colptr, rowind, perm) tuples."""
    probe = BatchCholesky(mats, amalg_max_zeros=8)
    inf = probe.info()
    return tune_config(lambda kw: BatchCholesky(mats, **kw), vals, inf["n"], inf["flops_alg"], B, precision, reps,
                       use_cache, **space)


def tune_single_config(n, colptr, rowind, perm, vals, B=None, precision="f64", reps: int = 5, use_cache=True,
                       **space):
    probe = SparseCholesky(n, colptr, rowind, perm, amalg_max_zeros=8)
    inf = probe.info()
    return tune_config(lambda kw: SparseCholesky(n, colptr, rowind, perm, **kw), vals, inf["n"], inf["flops_alg"],
                       B, precision, reps, use_cache, **space)
