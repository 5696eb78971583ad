"""The allocation-free solve (spchol_solve_noalloc) against spchol_solve,
called through the C ABI: two calls in a row on one GPU, the second with a
smaller matrix and fewer right-hand sides, each compared with the handle's
own solve of the same block and with the oracle's backward-error bar; a
size beyond the static workspace is rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def _solve_both(p, z, nrhs, seed):
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((nrhs, p.n))  # (nrhs, n): column-major n x nrhs
    lib = sc.lib()
    X1 = torch.tensor(B, device="cuda")
    X2 = torch.tensor(B, device="cuda")
    assert lib.spchol_solve_noalloc(F._h, C.c_void_p(X1.data_ptr()), nrhs, p.n, None) == 0, \
        lib.spchol_last_error()
    assert lib.spchol_solve(F._h, C.c_void_p(X2.data_ptr()), nrhs, p.n, None) == 0, lib.spchol_last_error()
    torch.cuda.synchronize()
    X1, X2 = X1.cpu().numpy(), X2.cpu().numpy()
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    eta1, _ = oracle.backward_error(A, X1.T, B.T)
    eta2, _ = oracle.backward_error(A, X2.T, B.T)
    d = np.abs(X1 - X2).max() / np.abs(X2).max()
    print(f"  n={p.n} nrhs={nrhs}: eta noalloc {eta1.max():.2e} eta solve {eta2.max():.2e} rel diff {d:.2e}",
          flush=True)
    assert eta1.max() <= 1e-12 and eta2.max() <= 1e-12
    # same kernels and launch order; ancestor rows take atomic adds, so
    # only the summation order may differ
    assert d <= 1e-12
    return S, F


def test_noalloc_solve_matches_solve_twice():
    print("noalloc: first call (3D 7-point 16^3, 6 right-hand sides)", flush=True)
    S1, F1 = _solve_both(gen.make_config(1, side=16), 8, 6, 1)
    print("noalloc: second call (2D 5-point 20^2, 2 right-hand sides)", flush=True)
    S2, F2 = _solve_both(gen.make_config(0, side=20), 0, 2, 2)
    # beyond the static workspace: rejected on the host, nothing enqueued
    big = 1 + (1 << 21) // S2.n
    Bt = torch.zeros((1, S2.n), dtype=torch.float64, device="cuda")
    rc = sc.lib().spchol_solve_noalloc(F2._h, C.c_void_p(Bt.data_ptr()), big, S2.n, None)
    assert rc == -1
    assert b"exceeds" in sc.lib().spchol_last_error()
