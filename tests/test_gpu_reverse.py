"""Reverse mode: selected inversion and the adjoints of logdet and of the
solve, against a dense inverse, torch dense autograd, the oracle's closed
forms and central finite differences.

Gate (the reverse-mode target): gradients match to 1e-6 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from conftest import gpu_available
from gpu_util import permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def _dense_spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    M = G @ G.T / n + np.eye(n)
    Ls = sp.csc_matrix(np.tril(M))
    Ls.sort_indices()
    return n, Ls.indptr.astype(np.int64), Ls.indices.astype(np.int64), Ls.data, rng.permutation(n)


CASES = {
    "cfg0_12": lambda: (lambda p: (p.n, p.colptr, p.rowind, p.vals, p.perm, 0))(gen.make_config(0, side=12)),
    "cfg1_10_z8": lambda: (lambda p: (p.n, p.colptr, p.rowind, p.vals, p.perm, 8))(gen.make_config(1, side=10)),
    "cfg2_5_z8": lambda: (lambda p: (p.n, p.colptr, p.rowind, p.vals, p.perm, 8))(gen.make_config(2, side=5)),
    "dense150": lambda: _dense_spd(150, 3) + (0,),
}


def _refined_inverse(C):
    """C^{-1} to about unit roundoff whatever kappa: the float64 inverse
    corrected twice by Z <- Z + Z (I - C Z), the residual I - C Z formed in
    extended precision (np.longdouble, 64-bit significand) from the exact
    float64 entries of C, one sparse row at a time."""
    Cs = sp.csr_matrix(C)
    Z = np.linalg.inv(C)
    for _ in range(2):
        Zl = Z.astype(np.longdouble)
        R = np.zeros(C.shape, dtype=np.longdouble)
        for i in range(C.shape[0]):
            a, b = Cs.indptr[i], Cs.indptr[i + 1]
            acc = np.zeros(C.shape[1], dtype=np.longdouble)
            acc[i] = 1.0
            for k, v in zip(Cs.indices[a:b], Cs.data[a:b]):
                acc -= np.longdouble(v) * Zl[k]
            R[i] = acc
        Z = Z + Z @ R.astype(np.float64)
    return Z


@pytest.mark.parametrize("name", list(CASES))
def test_selected_inverse_vs_dense(name):
    """Z on L's pattern against C^{-1}.  The reference is accurate to about
    unit roundoff u = 2^-53 (refined inverse), so the difference is the
    library's own error.  A backward-stable factorization (measured
    ||C - L L^T|| / ||C|| ~ u here) determines C^{-1} only to first order
    kappa(C) times that backward error, so the gate is max(1e-11, kappa u):
    1e-11 for the well-conditioned cases, kappa u (no safety factor) for the
    ill-conditioned 3D case."""
    n, cp, ri, vv, perm, z = CASES[name]()
    print(f"selinv case {name} n={n}", flush=True)
    S = sc.SparseCholesky(n, cp, ri, perm, 0, z)
    F = S.factor(torch.tensor(vv, device="cuda"))
    Zst = F.selinv().cpu().numpy()
    Zg, _ = storage_to_csc(S.export(), S.storage_offsets(), Zst, n)
    A = oracle.full_matrix(n, cp, ri, vv)
    Cm = permuted_matrix(A, np.asarray(perm)).toarray()
    Zd = _refined_inverse(Cm)
    Zg = Zg.tocoo()
    err = np.abs(Zg.data - Zd[Zg.row, Zg.col]).max() / np.abs(Zd).max()
    ev = np.linalg.eigvalsh(Cm)
    kappa = ev[-1] / ev[0]
    tol = max(1e-11, kappa * 2.0 ** -53)
    print(f"  max rel error on the pattern {err:.2e} (kappa {kappa:.1e}, tol {tol:.1e})", flush=True)
    assert err <= tol


def test_gradients_vs_torch_dense():
    p = gen.make_config(0, side=8)
    n = p.n
    S = sc.SparseCholesky(n, p.colptr, p.rowind, p.perm, 0, 0)
    v = torch.tensor(p.vals, device="cuda", requires_grad=True)
    b = torch.tensor(p.B[:, 0], device="cuda", requires_grad=True)
    rng = np.random.default_rng(5)
    c = torch.tensor(rng.standard_normal(n), device="cuda")
    ld, x = sc.logdet_solve(S, v, b)
    loss = 0.7 * ld + (c * x).sum()
    loss.backward()
    # dense reference on the CPU (float64)
    r, col = oracle.entry_coords(p.colptr, p.rowind)
    vc = torch.tensor(p.vals, dtype=torch.float64, requires_grad=True)
    bc = torch.tensor(p.B[:, 0], dtype=torch.float64, requires_grad=True)
    A = torch.zeros((n, n), dtype=torch.float64).index_put((torch.tensor(r), torch.tensor(col)), vc)
    A = A + A.T - torch.diag(torch.diagonal(A))
    lref = 0.7 * torch.logdet(A) + (c.cpu() * torch.linalg.solve(A, bc)).sum()
    lref.backward()
    np.testing.assert_allclose(v.grad.cpu().numpy(), vc.grad.numpy(), rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(b.grad.cpu().numpy(), bc.grad.numpy(), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("side", [12, 20])
def test_gradients_vs_oracle_closed_form(side):
    """GRF 3D recipe: Abar on 64 sampled entries against the oracle's closed
    forms (unit-vector solves), relative 1e-6."""
    p = gen.make_config(4, side=side)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    F = S.factor(torch.tensor(p.vals, device="cuda"))
    x = F.solve(torch.tensor(p.B[:, 0], device="cuda"))
    rng = np.random.default_rng(11)
    xbar = rng.standard_normal(p.n)
    g = 0.3
    Abar, Bbar = F.backward(x, torch.tensor(xbar, device="cuda"), g)
    Abar = Abar.cpu().numpy()
    osym = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    of = osym.factor(p.vals)
    ent = rng.choice(p.colptr[-1], size=64, replace=False)
    # include a few diagonal entries
    ent[:4] = p.colptr[rng.choice(p.n, 4, replace=False)]
    xo = of.solve(p.B[:, 0])
    gl = oracle.grad_logdet(of, p.colptr, p.rowind, ent)
    gs, lam = oracle.grad_solve(of, p.colptr, p.rowind, xo, xbar, ent)
    ref = g * gl + gs
    err = np.abs(Abar[ent] - ref) / np.maximum(np.abs(ref), 1e-300)
    print(f"  side {side}: max rel grad error {err.max():.2e}", flush=True)
    assert err.max() <= 1e-6
    np.testing.assert_allclose(Bbar.cpu().numpy(), lam.ravel(), rtol=1e-8, atol=1e-12 * np.abs(lam).max())


def test_finite_differences():
    """Central differences of l = c1 logdet + c2^T x on 16 entries."""
    p = gen.make_config(4, side=8)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    rng = np.random.default_rng(2)
    c1, c2 = 0.5, rng.standard_normal(p.n)
    bt = torch.tensor(p.B[:, 0], device="cuda")

    def loss(vals):
        F = S.factor(torch.tensor(vals, device="cuda"))
        x = F.solve(bt).cpu().numpy()
        return c1 * F.logdet() + c2 @ x

    F = S.factor(torch.tensor(p.vals, device="cuda"))
    x = F.solve(bt)
    Abar, _ = F.backward(x, torch.tensor(c2, device="cuda"), c1)
    Abar = Abar.cpu().numpy()
    ent = rng.choice(p.colptr[-1], size=16, replace=False)
    worst = 0.0
    for e in ent:
        h = 1e-5 * max(abs(p.vals[e]), 1e-3)
        vp = p.vals.copy(); vp[e] += h
        vm = p.vals.copy(); vm[e] -= h
        fd = (loss(vp) - loss(vm)) / (2 * h)
        worst = max(worst, abs(fd - Abar[e]) / max(abs(Abar[e]), 1e-8))
    print(f"  FD max rel error {worst:.2e}", flush=True)
    assert worst <= 1e-5


def test_selected_inverse_graph_replays():
    """On a stream of its own, repeated selected inversions go through the
    graph cache (eager, then captured, then replayed); every call, with
    other work and synchronizations between them, matches the first one
    (eager) to rounding (the Y blocks are summed with atomics)."""
    n, cp, ri, vv, perm, z = CASES["cfg1_10_z8"]()
    print(f"selinv graph replays n={n}", flush=True)
    S = sc.SparseCholesky(n, cp, ri, perm, 0, z)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        F = S.factor(torch.tensor(vv, device="cuda"))
        ref = F.selinv().clone()
        torch.cuda.synchronize()
        scale = ref.abs().max().item()
        B = torch.randn(3, n, dtype=torch.float64, device="cuda")
        for it in range(5):
            Z = F.selinv()
            torch.cuda.synchronize()
            err = (Z - ref).abs().max().item() / scale
            print(f"  call {it}: max rel difference {err:.2e}", flush=True)
            assert err <= 1e-12
            X = B.clone()
            F.solve_(X)  # other work between the calls
            torch.cuda.synchronize()
