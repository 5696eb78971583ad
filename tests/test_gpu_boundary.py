"""Boundary options on the GPU: the deterministic schedule (bitwise equal
runs), the workspace limit on the device paths, the pivot-failure injection
hook and the per-level trace."""
import json
import os

import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def _run_once(p, z, det):
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z, deterministic=det)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    X = F.solve(torch.tensor(p.B, device="cuda"))
    Z = F.selinv()
    torch.cuda.synchronize()
    return S, F.storage().cpu().numpy(), X.cpu().numpy(), F.logdet(), Z.cpu().numpy()


# (28^3: a root separator of 12-13 panels, past the window of the default
# schedule's panel rounds, which the deterministic schedule does without)
@pytest.mark.parametrize("cfg,side", [(1, 20), (2, 7), (0, 32), (1, 28)])
def test_deterministic_runs_are_bitwise_equal(cfg, side):
    p = gen.make_config(cfg, side=side)
    z = p.meta["amalg_z"]
    print(f"deterministic cfg={cfg} side={side} n={p.n}", flush=True)
    S, L1, X1, ld1, Z1 = _run_once(p, z, True)
    _, L2, X2, ld2, Z2 = _run_once(p, z, True)
    assert np.array_equal(L1.view(np.uint64), L2.view(np.uint64))
    assert np.array_equal(X1.view(np.uint64), X2.view(np.uint64))
    assert ld1 == ld2
    assert np.array_equal(Z1.view(np.uint64), Z2.view(np.uint64))
    # and it is the same factor as the oracle's
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    of = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z).factor(p.vals)
    Cm = permuted_matrix(A, p.perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), L1, p.n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    eta, _ = oracle.backward_error(A, X1, p.B)
    print(f"  bitwise equal; vs oracle frobenius {fro:.2e}, eta {eta.max():.2e}", flush=True)
    assert upper == 0.0 and offmax == 0.0 and fro <= 1e-12 and eta.max() <= 1e-12
    assert abs(ld1 - of.logdet()) <= 1e-12 * abs(of.logdet())
    # the default (atomic) schedule gives the same factor to rounding
    _, L3, X3, ld3, _ = _run_once(p, z, False)
    assert np.abs(L3 - L1).max() <= 1e-10 * np.abs(L1).max()


def test_workspace_limit_on_device_paths():
    p = gen.make_config(1, side=12)
    base = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    vals = torch.tensor(p.vals, device="cuda")
    # just what the factor needs: the factorization fits, a solve does not
    h = base.info()
    probe = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, workspace_limit=1)
    with pytest.raises(sc.SpcholError) as ei:
        probe.factor(vals)
    assert ei.value.status == -4
    need = int(str(ei.value).split("needs ")[1])
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, workspace_limit=need)
    F = S.factor(vals)
    with pytest.raises(sc.SpcholError) as ei:
        F.solve(torch.tensor(p.B, device="cuda"))
    assert ei.value.status == -4 and "workspace limit" in str(ei.value)
    # room for one right-hand side's work vectors (3 n doubles)
    S2 = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, workspace_limit=need + 24 * p.n)
    F2 = S2.factor(vals)
    x = F2.solve(torch.tensor(p.B[:, 0], device="cuda")).cpu().numpy()
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    eta, _ = oracle.backward_error(A, x, p.B[:, 0])
    assert eta.max() <= 1e-12
    with pytest.raises(sc.SpcholError):  # the selected inverse does not fit
        F2.selinv()
    assert h["storage"] > 0


def test_fail_at_hook_reports_a_pivot_failure(monkeypatch):
    p = gen.make_config(0, side=16)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm)
    vals = torch.tensor(p.vals, device="cuda")
    monkeypatch.setenv("SPCHOL_DEBUG_FAIL_AT", "37")
    with pytest.raises(sc.NotPositiveDefinite) as ei:
        S.factor(vals)
    assert ei.value.info == 37
    monkeypatch.delenv("SPCHOL_DEBUG_FAIL_AT")
    F = S.factor(vals)  # a fresh handle: the hook is read when launches are enqueued
    assert F.info == 0


def test_trace_prints_levels(monkeypatch, capfd):
    p = gen.make_config(1, side=12)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    monkeypatch.setenv("SPCHOL_TRACE", "1")
    S.factor(torch.tensor(p.vals, device="cuda"))
    monkeypatch.delenv("SPCHOL_TRACE")
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith('{"spchol_trace"')]
    assert lines, err
    tr = json.loads(lines[-1])
    assert tr["spchol_trace"] == "factor" and len(tr["levels"]) == S.info()["nlevels"]
    assert all(lv["launches"] >= 1 and lv["ms"] >= 0 for lv in tr["levels"])
