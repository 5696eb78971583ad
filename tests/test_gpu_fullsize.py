"""Parity at the benchmark's full size (64^3 7-point Laplacian, n = 262,144,
nested dissection, amalgamation z = 8), in the launch configuration that
bench.py times.

The whole oracle factorization takes minutes, so the checks are:
  * sampled columns: the first t = 32,768 columns form a complete nested
    dissection subtree; column j of L depends only on columns k < j, so the
    oracle's left-looking factorization stopped after t columns gives those
    columns exactly (up to rounding), compared entry by entry;
  * residual probes ||(C - L L^T) v|| / (||C||_F ||v||) on random v,
    computed on the host from the device factor;
  * the normwise backward error of the solve <= 1e-12.
Also a mid-size 3D case (40^3) compared in full.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def llt_probe(export, off, Lst, v):
    """L (L^T v) from supernodal storage (upper triangles of the diagonal
    blocks are stored zeros, so whole rectangles can be multiplied)."""
    spr, rp, ri = export["super_ptr"], export["row_ptr"], export["row_idx"]
    n = v.shape[0]
    w = np.zeros_like(v)
    blocks = []
    for J in range(len(spr) - 1):
        f, k = int(spr[J]), int(spr[J + 1] - spr[J])
        R = ri[rp[J]:rp[J + 1]]
        blk = Lst[off[J]:off[J] + k * len(R)].reshape(k, len(R)).T  # m x k
        blocks.append((f, k, R, blk))
        w[f:f + k] = blk.T @ v[R]
    out = np.zeros_like(v)
    for f, k, R, blk in blocks:
        out[R] += blk @ w[f:f + k]
    return out


def test_bench_config_fullsize():
    p = gen.make_config(1)
    z = p.meta["amalg_z"]
    print(f"fullsize: n={p.n} z={z}", flush=True)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    X = F.solve(torch.tensor(p.B, device="cuda")).cpu().numpy()
    Lst = F.storage().cpu().numpy()
    ld = F.logdet()
    torch.cuda.synchronize()
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    eta, comp = oracle.backward_error(A, X, p.B)
    print(f"  eta={eta.max():.3e} comp={comp.max():.3e} logdet={ld:.12e}", flush=True)
    assert eta.max() <= 1e-12
    e = S.export()
    off = S.storage_offsets()
    # residual probes
    Cm = permuted_matrix(A, p.perm)
    cnorm = sp.linalg.norm(Cm)
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(4):
        v = rng.standard_normal(p.n)
        r = Cm @ v - llt_probe(e, off, Lst, v)
        worst = max(worst, np.linalg.norm(r) / (cnorm * np.linalg.norm(v)))
    print(f"  residual probe {worst:.3e}", flush=True)
    assert worst <= 1e-12
    # sampled columns vs the oracle's prefix factorization
    t = 32768
    osym = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
    of = osym.factor(p.vals, ncols=t)
    assert of.info == 0
    Lo = of.L_csc()[:, :t]
    # GPU columns < t: supernodes entirely inside the prefix
    J_end = int(np.searchsorted(e["super_ptr"], t))
    assert e["super_ptr"][J_end] == t
    sub = dict(super_ptr=e["super_ptr"][:J_end + 1], row_ptr=e["row_ptr"][:J_end + 1], row_idx=e["row_idx"])
    Lg, upper = storage_to_csc(sub, off, Lst, p.n)
    assert upper == 0.0
    Lg = Lg[:, :t]
    elt, offmax, fro = compare_factor(Lg, Lo, Cm.diagonal())
    print(f"  prefix columns: elementwise {elt:.3e} frobenius {fro:.3e} offstruct {offmax}", flush=True)
    assert offmax == 0.0
    assert fro <= 1e-12
    assert elt <= 1e-11


def test_midsize_3d_full_compare():
    """40^3 with the 64^3 recipe: compared with the full oracle factor."""
    p = gen.make_config(1, side=40)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    Lst = F.storage().cpu().numpy()
    ld = F.logdet()
    X = F.solve(torch.tensor(p.B, device="cuda")).cpu().numpy()
    osym = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    of = osym.factor(p.vals)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    Cm = permuted_matrix(A, p.perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), Lst, p.n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    print(f"  40^3: elementwise {elt:.3e} frobenius {fro:.3e}", flush=True)
    assert upper == 0.0 and offmax == 0.0
    assert fro <= 1e-12
    eta, _ = oracle.backward_error(A, X, p.B)
    assert eta.max() <= 1e-12
    assert abs(ld - of.logdet()) <= 1e-12 * abs(of.logdet())
