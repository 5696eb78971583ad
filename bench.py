"""Benchmark of the supernodal Cholesky hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1]
                    [--no-cpu-baseline] [--no-extras] [--copy-probe MiB]

Headline (one step = the whole hot path on inputs already resident in device
memory, 3D 7-point 64^3 workload): value scatter, leaves-to-root supernodal
factorization (panel Cholesky, triangular solve, update + relative-index
scatter), the forward and backward supernodal solves and logdet.  The
symbolic analysis (host) runs once before timing.

value = algorithmic factorization flops (sum_j c_j^2 over the true column
counts) / mean factorization time, HIP events on the stream the kernels run
on.  The timed steps replay the factorization and the solve as captured
hipGraphs (the same kernels and task lists, one host launch each); an eager
pass before them, with a HIP event pair around every launch and every
launch running alone on one stream, gives the per-kernel breakdown
(`kernels`) and the roofline of the dominant kernel; a second eager pass,
with the far updates of each level on a second stream as in the graphs,
gives the eager times (`eager_*`) and the dominant kernel's launches as they
overlap (`roofline.overlapped`).  The same JSON line carries, measured in the
same run:
  mixed_ir  - 3D 27-point 3-dof 40^3, 8 RHS: fp64 factor+solve against
              fp32- and bf16-update factor + solve + iterative refinement
              to a normwise backward error <= 1e-12 (per-RHS errors and
              whether refinement converged within 10 iterations);
  fwd_bwd   - 3D 48^3 random-field workload: forward (factor + solve +
              logdet) and reverse (selected inversion + gradient) times;
  batch     - 512 independent grids, factor + 4-RHS solve as one hipGraph;
  variants  - the headline matrix analysed other ways and factored the same
              way: RLB updates (with and without partition refinement), the
              paper's greedy supernode merging (25 % cap), the deterministic
              schedule, the library's own nested dissection; and the
              host-resident factorization (supernodes below the paper's
              size threshold on the host, a 256 MiB device budget).

--copy-probe runs a plain device copy of the given size (the calibration
run for the hardware byte counters) and nothing else.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor GFLOP/s, FP64 vs mixed+IR at backward err <=1e-12; fwd+bwd time"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from the hardware counters
# (FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, scales from a plain 1 GiB copy;
# profiles/update_ext_grid3d_64.md), valid for the kernel source they were
# taken with: reported only while the source hash matches.
MEASURED_TRAFFIC = {"kernel": "update_ext", "bytes_per_launch": 391025388,
                    "update_source_sha256_16": "59602839d495b36f"}


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_baseline(p, z, ncols=65536):
    """The oracle (plain single-thread C left-looking factorization) on a
    bounded sample: the first `ncols` columns of the same elimination order,
    which form a complete nested-dissection subtree (columns < t depend only
    on columns < t); ncols >= n times the whole factorization."""
    import oracle
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
    t = min(ncols, p.n)
    t0 = time.perf_counter()
    f = s.factor(p.vals, ncols=t)
    dt = time.perf_counter() - t0
    assert f.info == 0
    fl = s.flops(t)
    what = "the whole factorization" if t == p.n else f"the first {t} columns (a complete ND subtree, " \
           f"{fl:.3e} of {s.flops():.3e} algorithmic flops)"
    return dict(value=fl / dt / 1e9, unit="GFLOP/s", cores=1, host_cores=_host_cores(), kind="oracle",
                seconds=dt,
                sample=f"left-looking factorization of {what} of the same matrix and ordering, "
                       f"{dt:.1f} s on 1 thread of {_host_cores()} host cores")


UPDATE_REGION = ("// update: C[i, c] -= sum_t", "// One-panel lookahead")


def update_source_sha(text):
    """sha256[:16] of the update kernel's source (from its header comment to
    the next kernel), or None when the anchors are missing."""
    import hashlib
    a, b = text.find(UPDATE_REGION[0]), text.find(UPDATE_REGION[1])
    if a < 0 or b < a:
        return None
    return hashlib.sha256(text[a:b].encode()).hexdigest()[:16]


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel`, or None when the
    kernel's source changed since the counters were taken."""
    with open(os.path.join(ROOT, "paper_2409_14009_amd", "csrc", "kernels.hip")) as f:
        sha = update_source_sha(f.read())
    t = MEASURED_TRAFFIC
    if kernel != t["kernel"] or sha is None or sha != t["update_source_sha256_16"]:
        return None
    return t["bytes_per_launch"]


def _timed_steps(steps, stream, phases):
    """Run `steps` iterations of the callables in `phases` (list of
    (name, fn)); an event is recorded on `stream` before and after each
    phase.  Returns {name: mean ms}."""
    import torch
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        evs[k][0].record(stream)
        for i, (_, fn) in enumerate(phases):
            fn()
            evs[k][i + 1].record(stream)
    torch.cuda.synchronize()
    return {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
            for i, (name, _) in enumerate(phases)}


WIDE_K = 256


def wide_update_levels(S, kmin=WIDE_K):
    """Levels of the schedule whose external-update work (tiled launches;
    the one-wavefront supernodes excluded) comes from supernodes of at
    least kmin columns on average, weighted by flops."""
    e = S.export()
    k = np.diff(np.asarray(e["super_ptr"])).astype(np.float64)
    m = np.diff(np.asarray(e["row_ptr"])).astype(np.float64)
    lev = np.asarray(e["level"])
    r = m - k
    small = (k <= 16) & (np.where(k <= 4, 4, 16) + m <= 64)
    w = np.where((r > 0) & ~small, k * r * (r + 1), 0.0)
    out = set()
    for lv in np.unique(lev):
        s = lev == lv
        if w[s].sum() > 0 and (w[s] * k[s]).sum() / w[s].sum() >= kmin:
            out.add(int(lv))
    return out


def headline(args, dev):
    import torch
    import gen
    import paper_2409_14009_amd as sc

    log(f"config {args.config} setup")
    p = gen.make_config(args.config, side=args.side)
    z = p.meta["amalg_z"]
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, p.meta["snode_mode"], z)
    info = S.info()
    vals = torch.tensor(p.vals, device=dev)
    Bt = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)  # (nrhs, n): column-major n x nrhs
    Xt = torch.empty_like(Bt)
    stream = torch.cuda.current_stream()

    F = S.factor(vals)
    for _ in range(args.warmup):
        F.refactor(vals)
        Xt.copy_(Bt)
        F.solve_(Xt)
        F.logdet()
    torch.cuda.synchronize()
    log(f"warmup done, timing {args.steps} steps")

    def eager_pass(alone):
        """steps eager factor + solve + logdet with an event pair around every
        launch; alone: each launch by itself on one stream"""
        F.profile(True, alone=alone)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            e0, e1, e2 = ev[k]
            e0.record(stream)
            F.refactor(vals)
            e1.record(stream)
            Xt.copy_(Bt)
            F.solve_(Xt)
            F.logdet()
            e2.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        recs = F.profile_launches()
        F.profile(False)
        return (recs, float(np.mean([a.elapsed_time(b) for a, b, _ in ev])),
                float(np.mean([b.elapsed_time(c) for _, b, c in ev])), (t1 - t0) * 1e3 / args.steps)

    # kernel figures from launches that each had the GPU to themselves (the
    # far updates otherwise share it with the near ones and the panel chain)
    recs, alone_factor_ms, _, _ = eager_pass(True)
    eta = F.berr_(vals, Bt, Xt)
    # the eager times, and the dominant kernel's launches, as they overlap
    recs_ov, factor_ms, solve_ms, ms_per_step = eager_pass(False)
    eta = eta + F.berr_(vals, Bt, Xt)
    gflops = info["flops_alg"] / (factor_ms * 1e-3) / 1e9

    def per_kind(rs):
        out = {}
        for r in rs:
            a = out.setdefault(r["kind"], dict(launches=0, ms=0.0, flops=0.0, bytes=0.0))
            a["launches"] += 1
            a["ms"] += r["ms"]
            a["flops"] += r["flops"]
            a["bytes"] += r["bytes"]
        for kname in ("fill", "scatter_a", "factor", "update_int", "update_ext"):
            out.setdefault(kname, dict(launches=0, ms=0.0, flops=0.0, bytes=0.0))
        return out

    prof, prof_ov = per_kind(recs), per_kind(recs_ov)

    # dominant kernel of the factorization: the one carrying most of its
    # algorithmic work (the external update: ~83% of the flops at 64^3);
    # the panel chain (diagonal blocks + row tiles + lookahead tiles) is
    # reported beside it, it is bound by the latency of its sequential
    # pivot sweeps rather than by a throughput roof
    fk = ["fill", "scatter_a", "factor", "update_int", "update_ext"]
    dom = max(fk, key=lambda k: prof[k]["flops"])
    d = prof[dom]
    pc = prof["factor"]
    chain = dict(bound="latency", kernel="factor", launches_per_step=pc["launches"] / args.steps,
                 ms_per_step=pc["ms"] / args.steps,
                 achieved_tflops=pc["flops"] / (pc["ms"] * 1e-3) / 1e12 if pc["ms"] > 0 else None,
                 frac_of_fp64_mfma=(pc["flops"] / (pc["ms"] * 1e-3) / 1e12) / PEAK_FP64_TFLOPS if pc["ms"] > 0 else None)
    if dom in ("update_int", "update_ext", "factor"):
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=achieved / PEAK_FP64_TFLOPS, traffic=None)
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=achieved / PEAK_HBM_GBS, traffic=None)
    roof["traffic"] = measured_traffic(dom)
    roof.update(kernel=dom, launches_per_step=d["launches"] / args.steps,
                avg_launch_us=d["ms"] * 1e3 / max(d["launches"], 1),
                flops_per_step=d["flops"] / args.steps, bytes_per_step=d["bytes"] / args.steps,
                timing="each launch alone on one stream (eager pass, per-launch HIP events)",
                alone_factor_ms=alone_factor_ms)
    # the same kernel's launches as they run in the overlapped schedule: the
    # far updates of a level beside its near updates and the next level's
    # panel chain, so a launch's duration includes time shared with those
    do = prof_ov[dom]
    if do["ms"] > 0:
        a_ov = (do["flops"] if roof["bound"] == "mfma" else do["bytes"]) / (do["ms"] * 1e-3)
        a_ov = a_ov / 1e12 if roof["bound"] == "mfma" else a_ov / 1e9
        roof["overlapped"] = dict(avg_launch_us=do["ms"] * 1e3 / max(do["launches"], 1), achieved=a_ov,
                                  frac=a_ov / roof["peak"])
    # the large-supernode updates: external-update launches of the levels
    # whose update work comes from supernodes of >= 256 columns on average
    # (flop-weighted), the part the fp64 matrix cores can run near their peak
    wl = wide_update_levels(S)
    wr = [r for r in recs if r["kind"] == "update_ext" and r["level"] in wl]
    wms, wfl = sum(r["ms"] for r in wr), sum(r["flops"] for r in wr)
    wide = dict(min_avg_columns=WIDE_K, levels=len(wl), launches_per_step=len(wr) / args.steps,
                ms_per_step=wms / args.steps,
                share_of_update_flops=wfl / prof["update_ext"]["flops"] if prof["update_ext"]["flops"] else None,
                achieved=wfl / (wms * 1e-3) / 1e12 if wms > 0 else None, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                frac=wfl / (wms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS if wms > 0 else None)
    kernels = {k: dict(launches=v["launches"] / args.steps, ms=v["ms"] / args.steps,
                       gflops=(v["flops"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["flops"] else None,
                       gbs=(v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] else None)
               for k, v in prof.items() if v["launches"]}
    cfg = {
        "workload": p.meta["doc"],
        "n": p.n, "nnz_l": info["nnz_l"], "storage": info["storage"], "nsuper": info["nsuper"],
        "levels": info["nlevels"], "flops_alg": info["flops_alg"], "flops_exec": info["flops_exec"],
        "amalg_max_zeros": z, "nrhs": int(p.B.shape[1]), "seed": p.meta["seed"],
        "parallelism": "single GPU",
    }
    # The timed steps: the same launch sequences captured once as hipGraphs
    # (factorization; solve of Xt in place) and replayed, one host launch
    # each instead of one per task list.
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        Gf = F.capture(vals, stream=gs)
        Gs = F.capture(None, Xt, stream=gs)
        box = {}

        def solve_logdet():
            Xt.copy_(Bt)
            Gs.replay(gs)
            box["ld"] = F.logdet(stream=gs)

        for _ in range(args.warmup):
            Gf.replay(gs)
            solve_logdet()
        log(f"graph warmup done, timing {args.steps} steps")
        t0 = time.perf_counter()
        tg = _timed_steps(args.steps, gs, [("factor", lambda: Gf.replay(gs)), ("solve", solve_logdet)])
        t1 = time.perf_counter()
        gstatus = F.status(gs)
    eta_g = F.berr_(vals, Bt, Xt)
    Gf.close()
    Gs.close()
    if gstatus != 0:
        raise RuntimeError(f"factorization reported a non-positive pivot at column {gstatus}")
    value = info["flops_alg"] / (tg["factor"] * 1e-3) / 1e9
    res = dict(value=value, ms_per_step=(t1 - t0) * 1e3 / args.steps, factor_ms=tg["factor"], panel_chain=chain,
               wide_updates=wide,
               solve_logdet_ms=tg["solve"], eager_factor_ms=factor_ms, eager_solve_logdet_ms=solve_ms,
               eager_ms_per_step=ms_per_step, eager_gflops=gflops,
               backward_error=max(max(eta), max(eta_g)), logdet=box["ld"], roofline=roof, kernels=kernels,
               config=cfg)
    del F
    return res, p, z


def mixed_ir(args, dev):
    """fp64 factor + solve vs fp32-update factor + solve + refinement."""
    import torch
    import gen
    import paper_2409_14009_amd as sc

    log("mixed precision setup (3D 27-point 3-dof 40^3, 8 RHS)")
    p = gen.make_config(2)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, p.meta["snode_mode"], p.meta["amalg_z"])
    info = S.info()
    vals = torch.tensor(p.vals, device=dev)
    Bt = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)
    Xt = torch.empty_like(Bt)
    # a stream of its own (default priority): repeated factorizations and
    # solves with the same arguments replay captured graphs, for both forms
    stream = torch.cuda.Stream()
    steps = max(2, args.steps // 2)
    with torch.cuda.stream(stream):
        return _mixed_ir_body(args, p, S, info, vals, Bt, Xt, stream, steps)


# dense matrix-core peaks of the update products by precision (TFLOP/s)
PEAK_UPDATE_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


def _update_roofline(F, S, vals, prec):
    """One eager factorization with per-launch events, each launch alone on
    one stream: the external update's
    algorithmic rate against the matrix-core peak of its product precision,
    all levels and the wide-supernode levels."""
    F.profile(True, alone=True)
    F.refactor(vals, precision=prec)
    recs = F.profile_launches()
    F.profile(False)
    peak = PEAK_UPDATE_TFLOPS[prec]
    up = [r for r in recs if r["kind"] == "update_ext"]
    wl = wide_update_levels(S)
    wr = [r for r in up if r["level"] in wl]

    def rate(rs):
        ms, fl = sum(r["ms"] for r in rs), sum(r["flops"] for r in rs)
        a = fl / (ms * 1e-3) / 1e12 if ms > 0 else None
        return dict(launches=len(rs), ms=ms, achieved=a, frac=a / peak if a is not None else None)

    return dict(precision=prec, peak=peak, unit="TFLOP/s", all=rate(up), wide=rate(wr))


def _mixed_ir_body(args, p, S, info, vals, Bt, Xt, stream, steps):
    F = S.factor(vals)
    for _ in range(args.warmup):
        F.refactor(vals)
        Xt.copy_(Bt)
        F.solve_(Xt)
    t64 = _timed_steps(steps, stream, [("factor", lambda: F.refactor(vals)),
                                       ("solve", lambda: (Xt.copy_(Bt), F.solve_(Xt)))])
    eta64 = F.berr_(vals, Bt, Xt)
    roof64 = _update_roofline(F, S, vals, "f64")
    del F
    out = dict(workload=p.meta["doc"], n=p.n, nrhs=int(p.B.shape[1]), flops_alg=info["flops_alg"],
               fp64=dict(factor_ms=t64["factor"], factor_solve_ms=t64["factor"] + t64["solve"],
                         gflops=info["flops_alg"] / t64["factor"] * 1e-6, berr=eta64, update_roofline=roof64))
    for prec in ("f32", "bf16"):
        Fm = S.factor(vals, precision=prec)
        it_box = {}

        def refine():
            berr, it = Fm.refine_(vals, Bt, Xt, tol=1e-12, max_iter=10, check=False)
            it_box["berr"], it_box["it"] = berr, it

        for _ in range(args.warmup):
            Fm.refactor(vals, precision=prec)
            refine()
        tm = _timed_steps(steps, stream, [("factor", lambda: Fm.refactor(vals, precision=prec)),
                                          ("solve_ir", refine)])
        total = tm["factor"] + tm["solve_ir"]
        ok = bool(max(it_box["berr"]) <= 1e-12)
        roof = _update_roofline(Fm, S, vals, prec)
        out[prec + "_ir"] = dict(factor_ms=tm["factor"], solve_ir_ms=tm["solve_ir"], total_ms=total,
                                 gflops=info["flops_alg"] / tm["factor"] * 1e-6, iterations=it_box["it"],
                                 path="pcg" if Fm.last_refine_path else "ir", converged=ok, berr=it_box["berr"],
                                 speedup_vs_fp64=out["fp64"]["factor_solve_ms"] / total if ok else None,
                                 update_roofline=roof)
        del Fm
    return out


def fwd_bwd(args, dev):
    """Forward (factor + solve + logdet) and reverse (gradients of logdet
    and of x = A^-1 b w.r.t. A's values and b) on the 48^3 workload."""
    import torch
    import gen
    import paper_2409_14009_amd as sc

    log("reverse mode setup (3D 48^3 random field)")
    p = gen.make_config(4)
    vals = torch.tensor(p.vals, device=dev)
    Bt = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)
    Xt = torch.empty_like(Bt)
    rng = np.random.default_rng(p.meta["seed"] + 1)
    Xbar = torch.tensor(rng.standard_normal(p.n), device=dev)
    # a stream of its own (default priority), so that the repeated
    # factorization and solve replay captured graphs
    stream = torch.cuda.Stream()
    steps = max(2, args.steps // 2)
    # the workload's analysis (the paper's greedy merging), and the
    # per-column zero cap z = 8 beside it
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, p.meta["snode_mode"], p.meta["amalg_z"],
                          amalg_rule=p.meta["amalg_rule"], amalg_cap_percent=p.meta["amalg_cap_percent"])
    with torch.cuda.stream(stream):
        out = _fwd_bwd_body(args, p, S, S.info(), vals, Bt, Xt, Xbar, stream, steps)
    del S
    S8 = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, p.meta["snode_mode"], 8)
    with torch.cuda.stream(stream):
        o8 = _fwd_bwd_body(args, p, S8, S8.info(), vals, Bt, Xt, Xbar, stream, steps)
    out["amalgamation"] = "greedy merging, 25 % cap" if p.meta["amalg_rule"] == 1 else f"z={p.meta['amalg_z']}"
    out["with_z8"] = {k: o8[k] for k in ("fwd_ms", "bwd_ms", "fwd_bwd_ms", "grads_finite")}
    return out


def _fwd_bwd_body(args, p, S, info, vals, Bt, Xt, Xbar, stream, steps):
    import torch
    F = S.factor(vals)
    box = {}

    def fwd():
        F.refactor(vals)
        Xt.copy_(Bt)
        F.solve_(Xt)
        box["ld"] = F.logdet()

    def bwd():
        box["g"] = F.backward(Xt.view(-1), Xbar, 1.0)

    for _ in range(args.warmup):
        fwd()
        bwd()
    t = _timed_steps(steps, stream, [("fwd", fwd), ("bwd", bwd)])
    Abar, Bbar = box["g"]
    ok = bool(torch.isfinite(Abar).all().item() and torch.isfinite(Bbar).all().item())
    return dict(workload=p.meta["doc"], n=p.n, flops_alg=info["flops_alg"], fwd_ms=t["fwd"], bwd_ms=t["bwd"],
                fwd_bwd_ms=t["fwd"] + t["bwd"], grads_finite=ok, logdet=box["ld"])


def batch(args, dev):
    """512 independent grids: factor + 4-RHS solve captured in one hipGraph,
    with the analysis (supernode granularity, panel width, update method)
    chosen by the autotuner, and the untuned default beside it."""
    import torch
    import gen
    import scipy.sparse as sp
    import paper_2409_14009_amd as sc
    from paper_2409_14009_amd import autotune

    log("batch setup (512 grids)")
    probs = gen.make_batch()
    z = probs[0].meta["amalg_z"]
    mats = [(q.n, q.colptr, q.rowind, q.perm) for q in probs]
    vals = torch.tensor(np.concatenate([q.vals for q in probs]), device=dev)
    B0 = torch.tensor(np.ascontiguousarray(np.concatenate([q.B.T for q in probs], axis=1)), device=dev)
    X = torch.empty_like(B0)
    mats_a = [sp.csc_matrix((q.vals, q.rowind, q.colptr), shape=(q.n, q.n)) for q in probs]
    mats_a = [A + sp.tril(A, -1).T for A in mats_a]

    def run(S, precision):
        """factor + 4-RHS solve as one graph replay; per-matrix normwise
        backward error of the result (fp64, host)"""
        cnt, co, _ = S.batch_info()
        F = S.factor(vals, precision=precision)
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            G = F.capture(vals, X, stream=gs)
            for _ in range(args.warmup + 1):
                X.copy_(B0)
                G.replay(gs)
            steps = max(5, args.steps)
            t = _timed_steps(steps, gs, [("reset", lambda: X.copy_(B0)), ("graph", lambda: G.replay(gs))])
            status = F.status(gs)
        gs.synchronize()
        Xh = X.cpu().numpy()
        worst = 0.0
        for b, q in enumerate(probs):
            A = mats_a[b]
            x = Xh[:, co[b]:co[b + 1]].T
            r = q.B - A @ x
            an = abs(A).sum(axis=1).max()
            eta = np.abs(r).max(axis=0) / (an * np.abs(x).max(axis=0) + np.abs(q.B).max(axis=0))
            worst = max(worst, float(eta.max()))
        G.close()
        del F
        return t["graph"], status, worst

    S0 = sc.BatchCholesky(mats, amalg_max_zeros=z)
    info0 = S0.info()
    cnt = S0.batch_info()[0]
    ms_def, st_def, w_def = run(S0, "f64")
    del S0
    log("batch autotuning (granularity, panel width, update method)")
    t0 = time.perf_counter()
    cfg, times = autotune.tune_batch_config(mats, vals, B0, "f64", reps=3, use_cache=False)
    tune_s = time.perf_counter() - t0
    kw = autotune.config_kwargs(cfg)
    S = sc.BatchCholesky(mats, **kw)
    info = S.info()
    ms64, st64, w64 = run(S, "f64")
    ms32, st32, w32 = run(S, "f32")
    return dict(workload=gen.CONFIG_DOC[3], matrices=cnt, n_total=int(info["n"]), flops_alg=info["flops_alg"],
                tuned=dict(config=dict(amalg=list(cfg["amalg"]), panel_width=cfg["panel_width"],
                                       update=cfg["update"]), tuning_s=tune_s,
                           candidates_ms={k: v * 1e3 for k, v in times.items()}, nsuper=info["nsuper"],
                           levels=info["nlevels"], flops_exec=info["flops_exec"]),
                graph_ms=ms64, gflops=info["flops_alg"] / ms64 * 1e-6, matrices_per_s=cnt / (ms64 * 1e-3),
                status=st64, worst_berr=w64,
                untuned=dict(amalg_max_zeros=z, panel_width=64, update="rl", nsuper=info0["nsuper"],
                             levels=info0["nlevels"], graph_ms=ms_def, status=st_def, worst_berr=w_def),
                f32=dict(note="fp32 update products, fp64 diagonal blocks and solves, no refinement; tuned config",
                         graph_ms=ms32, matrices_per_s=cnt / (ms32 * 1e-3), status=st32, worst_berr=w32))


def copy_probe(mib):
    """A plain device copy of `mib` MiB, three times: the reference for the
    hardware byte counters (read + write of the buffer per dispatch)."""
    import torch
    n = (mib << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8}), flush=True)


def variants(args, dev, p, z):
    """Other analyses of the headline matrix, each factored through a
    captured graph: RLB update (with partition refinement), the paper's
    greedy supernode merging (25 % cap), the deterministic schedule, and
    the library's own nested dissection with the greedy merging."""
    import torch
    import paper_2409_14009_amd as sc

    log("variants of the headline analysis")
    vals = torch.tensor(p.vals, device=dev)
    Bt = torch.tensor(np.ascontiguousarray(p.B.T), device=dev)
    t0 = time.perf_counter()
    nd = sc.order_nd(p.n, p.colptr, p.rowind)
    order_s = time.perf_counter() - t0
    cases = [
        ("rlb_pr", p.perm, dict(amalg_max_zeros=z, update_method="rlb", partition_refinement=True)),
        ("rlb", p.perm, dict(amalg_max_zeros=z, update_method="rlb")),
        ("greedy25", p.perm, dict(amalg_rule=1, amalg_cap_percent=25)),
        ("deterministic", p.perm, dict(amalg_max_zeros=z, deterministic=True)),
        ("own_nd_greedy25", nd, dict(amalg_rule=1, amalg_cap_percent=25)),
    ]
    out = {"own_nd_order_s": order_s}
    for name, perm, kw in cases:
        t0 = time.perf_counter()
        S = sc.SparseCholesky(p.n, p.colptr, p.rowind, perm, 0, **kw)
        an_s = time.perf_counter() - t0
        info = S.info()
        F = S.factor(vals)
        gs = torch.cuda.Stream()
        with torch.cuda.stream(gs):
            G = F.capture(vals, stream=gs)
            for _ in range(args.warmup):
                G.replay(gs)
            t = _timed_steps(max(3, args.steps // 2), gs, [("factor", lambda: G.replay(gs))])
            st = F.status(gs)
        G.close()
        Xt = Bt.clone()
        F.solve_(Xt)
        eta = F.berr_(vals, Bt, Xt)
        out[name] = dict(analysis_s=an_s, nsuper=info["nsuper"], nnz_l=info["nnz_l"], storage=info["storage"],
                         flops_alg=info["flops_alg"], flops_exec=info["flops_exec"], factor_ms=t["factor"],
                         gflops=info["flops_alg"] / (t["factor"] * 1e-3) / 1e9, status=st,
                         backward_error=max(eta))
        log(f"  {name}: factor {t['factor']:.2f} ms")
        del F, S
        torch.cuda.empty_cache()
    # the host-resident factorization (the paper's architecture): supernodes
    # with k m below the paper's RL threshold on the host, the others on the
    # device within a 256 MiB budget, update blocks assembled by the host
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    info = S.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lh, st_info, st = S.factor_streamed(p.vals, device_budget=256 << 20, host_threshold=600000)
    dt = time.perf_counter() - t0
    Ld = S.factor(vals).storage().cpu().numpy()
    out["streamed"] = dict(host_threshold=600000, device_budget=256 << 20, seconds=dt,
                           gflops=info["flops_alg"] / dt / 1e9, status=st_info,
                           max_rel_diff_vs_device=float(np.abs(Ld - Lh).max() / np.abs(Ld).max()), **st)
    log(f"  streamed: {dt:.2f} s ({st['gpu_supernodes']} supernodes on the device, {st['host_supernodes']} on the host)")
    del Lh, Ld, S
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--side", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="time the oracle on the whole headline factorization (about a minute) and exit")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    if args.cpu_baseline_full:
        import gen
        p = gen.make_config(args.config, side=args.side)
        log("cpu baseline: the whole factorization")
        print(json.dumps({"cpu_baseline_full": cpu_baseline(p, p.meta["amalg_z"], ncols=p.n)}), flush=True)
        return
    res, p, z = headline(args, dev)
    extras = {}
    if not args.no_extras:
        extras["mixed_ir"] = mixed_ir(args, dev)
        torch.cuda.empty_cache()
        extras["fwd_bwd"] = fwd_bwd(args, dev)
        torch.cuda.empty_cache()
        extras["batch"] = batch(args, dev)
        torch.cuda.empty_cache()
        extras["variants"] = variants(args, dev, p, z)
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        cpu = cpu_baseline(p, z)

    out = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": res["config"],
        "factor_ms": res["factor_ms"],
        "eager_factor_ms": res["eager_factor_ms"],
        "eager_solve_logdet_ms": res["eager_solve_logdet_ms"],
        "eager_gflops": res["eager_gflops"],
        "solve_logdet_ms": res["solve_logdet_ms"],
        "backward_error": res["backward_error"],
        "logdet": res["logdet"],
        "roofline": res["roofline"],
        "panel_chain": res["panel_chain"],
        "wide_updates": res["wide_updates"],
        "cpu_baseline": cpu,
        "kernels": res["kernels"],
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
