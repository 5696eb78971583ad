"""Benchmark: numeric factorization (+ solve + logdet) of the 64^3 workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 1]
                    [--no-cpu-baseline]

One step = the whole hot path on inputs already resident in device memory:
value scatter, leaves-to-root supernodal factorization (panel Cholesky,
triangular solve, update + relative-index scatter), the forward and backward
supernodal solves of the right-hand side, and logdet.  The symbolic analysis
(host) runs once before timing.  Prints one JSON line.

value = algorithmic factorization flops (sum_j c_j^2 over the true column
counts) / mean factorization time measured with HIP events on the stream the
kernels run on.
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


def cpu_baseline(p, z, ncols=32768):
    """The oracle (plain single-thread C left-looking factorization) on a
    bounded sample: the first `ncols` columns of the same elimination order,
    which form a complete nested-dissection subtree (columns < t depend only
    on columns < t)."""
    import oracle
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
    t = min(ncols, p.n)
    t0 = time.perf_counter()
    f = s.factor(p.vals, ncols=t)
    dt = time.perf_counter() - t0
    assert f.info == 0
    fl = s.flops(t)
    return dict(value=fl / dt / 1e9, unit="GFLOP/s", cores=1, kind="oracle",
                sample=f"left-looking factorization of the first {t} columns (a complete ND subtree, "
                       f"{fl:.3e} of {s.flops():.3e} algorithmic flops) of the same matrix and ordering, "
                       f"{dt:.1f} s on 1 thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--side", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the sharded design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2409_14009_amd as sc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"bench: config {args.config} setup", file=sys.stderr, flush=True)
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
    print(f"bench: warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)

    F.profile(True)
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
        logdet = F.logdet()
        e2.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = F.profile_read()
    F.profile(False)
    factor_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    solve_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    gflops = info["flops_alg"] / (factor_ms * 1e-3) / 1e9

    # correctness of the timed result: normwise backward error of the solve
    import oracle
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    X = Xt.cpu().numpy().T
    eta, _ = oracle.backward_error(A, X, p.B)

    # dominant kernel of the factorization by summed event time
    fk = ["fill", "scatter_a", "factor", "update_int", "update_ext"]
    dom = max(fk, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    if dom in ("update_int", "update_ext", "factor"):
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = dict(bound="mfma", achieved=achieved, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=achieved / PEAK_FP64_TFLOPS, traffic=None)
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=achieved / PEAK_HBM_GBS, traffic=None)
    roof.update(kernel=dom, launches_per_step=d["launches"] / args.steps,
                avg_launch_us=d["ms"] * 1e3 / max(d["launches"], 1),
                flops_per_step=d["flops"] / args.steps, bytes_per_step=d["bytes"] / args.steps)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(p, z)

    kernels = {k: dict(launches=v["launches"] / args.steps, ms=v["ms"] / args.steps,
                       gflops=(v["flops"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["flops"] else None,
                       gbs=(v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] else None)
               for k, v in prof.items() if v["launches"]}
    out = {
        "metric": METRIC,
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": p.meta["doc"],
            "n": p.n, "nnz_l": info["nnz_l"], "storage": info["storage"], "nsuper": info["nsuper"],
            "levels": info["nlevels"], "flops_alg": info["flops_alg"], "flops_exec": info["flops_exec"],
            "amalg_max_zeros": z, "nrhs": int(p.B.shape[1]), "seed": p.meta["seed"],
            "parallelism": "single GPU",
        },
        "factor_ms": factor_ms,
        "solve_logdet_ms": solve_ms,
        "backward_error": float(eta.max()),
        "logdet": logdet,
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
