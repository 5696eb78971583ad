"""Parity of the three extra forms at their benchmark sizes, in the launch
configuration bench.py times.

  * 40^3 27-point stencil with 3 dofs per node (n = 192,000), 8 right-hand
    sides: the fp64 factor against the oracle on a prefix of complete
    columns (column j of L depends only on columns k < j), and the fp32- and
    bf16-update factors refined against the fp64 matrix, every right-hand
    side at a host-computed normwise backward error <= 1e-12 (the same
    quantity the library reports, recomputed here from A alone);
  * 512 independent grids (2D side U{12..48}, 3D side U{8..20}), 4 right-hand
    sides: every matrix's log-determinant against the oracle (relative
    1e-12) and every solve at a host backward error <= 1e-12 (fp64); the
    fp32-update variant reports its backward error and refines to 1e-12;
  * 48^3 random-field Laplacian (n = 110,592): reverse mode on 64 sampled
    stored entries against the oracle's closed forms (relative 1e-6), the
    adjoint of the right-hand side against the oracle's adjoint solve, and
    central finite differences on 64 entries of the loss
    c1 logdet(A) + c2^T A^{-1} b.
"""
import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


@pytest.fixture(scope="module")
def elasticity():
    p = gen.make_config(2)
    print(f"40^3x3: n={p.n} nnz_lower={p.colptr[-1]} nrhs={p.B.shape[1]}", flush=True)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, p.meta["amalg_z"])
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    return p, S, A


def test_elasticity_fp64_prefix_vs_oracle(elasticity):
    p, S, A = elasticity
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals)
    X = F.solve(torch.tensor(p.B, device="cuda")).cpu().numpy()
    Lst = F.storage().cpu().numpy()
    eta, _ = oracle.backward_error(A, X, p.B)
    print(f"  fp64 eta per rhs {np.array2string(eta, precision=2)}", flush=True)
    assert eta.max() <= 1e-12
    # the largest supernode boundary whose leading columns the oracle
    # factors in a few seconds
    z = p.meta["amalg_z"]
    osym = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
    e = S.export()
    spr = e["super_ptr"]
    t = 0
    for b in spr[1:]:
        if osym.flops(int(b)) > 6e10:
            break
        t = int(b)
    assert t >= p.n // 8
    of = osym.factor(p.vals, ncols=t)
    assert of.info == 0
    J_end = int(np.searchsorted(spr, t))
    sub = dict(super_ptr=spr[:J_end + 1], row_ptr=e["row_ptr"][:J_end + 1], row_idx=e["row_idx"])
    Lg, upper = storage_to_csc(sub, S.storage_offsets(), Lst, p.n)
    Cm = permuted_matrix(A, p.perm)
    elt, offmax, fro = compare_factor(Lg[:, :t], of.L_csc()[:, :t], Cm.diagonal())
    print(f"  prefix of {t} columns: elementwise {elt:.2e} frobenius {fro:.2e}", flush=True)
    assert upper == 0.0 and offmax == 0.0
    assert fro <= 1e-12 and elt <= 1e-11


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_elasticity_mixed_refined_host_eta(elasticity, prec):
    p, S, A = elasticity
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals, precision=prec)
    X, berr, it = F.refine(vals, torch.tensor(p.B, device="cuda"), tol=1e-12, max_iter=20)
    eta, comp = oracle.backward_error(A, X.cpu().numpy(), p.B)
    print(f"  {prec}: corrections {it} path {F.last_refine_path} host eta {np.array2string(eta, precision=2)} "
          f"componentwise max {comp.max():.2e}", flush=True)
    assert eta.shape == (8,)
    assert np.all(eta <= 1e-12)
    np.testing.assert_allclose(berr, eta, rtol=0.5, atol=2e-16)


def _check_batch(probs, co, lds, X, tol_eta):
    worst_ld = worst_eta = 0.0
    for b, q in enumerate(probs):
        o = oracle.Symbolic(q.n, q.colptr, q.rowind, q.perm, 0, 0).factor(q.vals)
        assert o.info == 0
        ldo = o.logdet()
        rel = abs(lds[b] - ldo) / max(abs(ldo), 1.0)
        eta, _ = oracle.backward_error(oracle.full_matrix(q.n, q.colptr, q.rowind, q.vals),
                                       X[:, co[b]:co[b + 1]].T, q.B)
        worst_ld, worst_eta = max(worst_ld, rel), max(worst_eta, float(eta.max()))
        assert rel <= 1e-12, (b, lds[b], ldo)
        assert eta.max() <= tol_eta, (b, eta)
    return worst_ld, worst_eta


def test_batch_512_every_matrix():
    probs = gen.make_batch()
    assert len(probs) == 512
    mats = [(q.n, q.colptr, q.rowind, q.perm) for q in probs]
    vals = np.concatenate([q.vals for q in probs])
    Bt = np.ascontiguousarray(np.concatenate([q.B.T for q in probs], axis=1))  # (4, N)
    print(f"batch: 512 matrices, N={Bt.shape[1]}, nrhs={Bt.shape[0]}", flush=True)
    S = sc.BatchCholesky(mats, amalg_max_zeros=8)
    cnt, co, _ = S.batch_info()
    assert cnt == 512
    v = torch.tensor(vals, device="cuda")
    B0 = torch.tensor(Bt, device="cuda")
    # fp64, through a captured graph as the bench runs it
    F = S.factor(v)
    Xg = torch.empty_like(B0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        G = F.capture(v, Xg, stream=stream)
        Xg.copy_(B0)
        G.replay(stream)
        lds = F.logdet_batch(stream=stream)
        assert F.status(stream) == 0
    stream.synchronize()
    w = _check_batch(probs, co, lds.cpu().numpy(), Xg.cpu().numpy(), 1e-12)
    print(f"  fp64: worst logdet rel {w[0]:.2e}, worst eta {w[1]:.2e}", flush=True)
    G.close()
    # fp32 update products: unrefined backward error reported, then refined
    F32 = S.factor(v, precision="f32")
    X32 = F32.solve_(B0.clone()).cpu().numpy()
    worst32 = 0.0
    for b, q in enumerate(probs):
        eta, _ = oracle.backward_error(oracle.full_matrix(q.n, q.colptr, q.rowind, q.vals),
                                       X32[:, co[b]:co[b + 1]].T, q.B)
        worst32 = max(worst32, float(eta.max()))
    Xr, berr, it = F32.refine(v, B0.t())
    Xr = Xr.t().contiguous().cpu().numpy()
    worst_r = 0.0
    for b, q in enumerate(probs):
        eta, _ = oracle.backward_error(oracle.full_matrix(q.n, q.colptr, q.rowind, q.vals),
                                       Xr[:, co[b]:co[b + 1]].T, q.B)
        worst_r = max(worst_r, float(eta.max()))
    print(f"  fp32 updates: unrefined worst eta {worst32:.2e}; refined ({it} corrections) {worst_r:.2e}",
          flush=True)
    assert worst32 <= 1e-6
    assert worst_r <= 1e-12


@pytest.fixture(scope="module")
def grf():
    p = gen.make_config(4)
    print(f"48^3 random field: n={p.n} nnz_lower={p.colptr[-1]}", flush=True)
    rule = dict(amalg_rule=p.meta["amalg_rule"], amalg_cap_percent=p.meta["amalg_cap_percent"])
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, p.meta["amalg_z"], **rule)
    osym = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, p.meta["amalg_z"], **rule)
    assert S.info()["nsuper"] == osym.nsuper
    of = osym.factor(p.vals)
    assert of.info == 0
    return p, S, of


def test_grf_reverse_64_entries_vs_closed_form(grf):
    p, S, of = grf
    vals = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals)
    x = F.solve(torch.tensor(p.B[:, 0], device="cuda"))
    rng = np.random.default_rng(64)
    xbar = rng.standard_normal(p.n)
    g = 0.7
    Abar, Bbar = F.backward(x, torch.tensor(xbar, device="cuda"), g)
    Abar = Abar.cpu().numpy()
    ent = rng.choice(p.colptr[-1], size=64, replace=False)
    ent[:8] = p.colptr[rng.choice(p.n, 8, replace=False)]  # some diagonal entries
    xo = of.solve(p.B[:, 0])
    gl = oracle.grad_logdet(of, p.colptr, p.rowind, ent)
    gs, lam = oracle.grad_solve(of, p.colptr, p.rowind, xo, xbar, ent)
    ref = g * gl + gs
    err = np.abs(Abar[ent] - ref) / np.abs(ref)
    print(f"  64 entries: max rel error {err.max():.2e} (median {np.median(err):.1e})", flush=True)
    assert err.max() <= 1e-6
    lam = lam.ravel()
    lerr = np.abs(Bbar.cpu().numpy() - lam).max() / np.abs(lam).max()
    print(f"  bbar max rel error {lerr:.2e}", flush=True)
    assert lerr <= 1e-8


def test_grf_finite_differences_64_entries(grf):
    """l(a) = c1 logdet(A) + c2^T A^{-1} b; central differences with
    h = 1e-3 max(|a_e|, 1e-3).  The quotient's truncation error is of
    relative order (h Z)^2 <= 1e-7 here (|a_e| Z_ii <= 1 for this
    diagonally dominant matrix); its rounding error is about eps |l| / h,
    which a smaller step would raise above the gate.  Each entry is gated
    at 1e-5 relative plus 64 eps |l| / h."""
    p, S, _ = grf
    rng = np.random.default_rng(65)
    c1, c2 = 0.5, rng.standard_normal(p.n)
    bt = torch.tensor(p.B[:, 0], device="cuda")
    vals0 = torch.tensor(p.vals, device="cuda")
    F = S.factor(vals0)

    def loss(v):
        F.refactor(v)
        x = F.solve(bt).cpu().numpy()
        return c1 * F.logdet() + float(c2 @ x)

    F.refactor(vals0)
    x = F.solve(bt)
    Abar, _ = F.backward(x, torch.tensor(c2, device="cuda"), c1)
    Abar = Abar.cpu().numpy()
    l0 = loss(vals0)
    ent = rng.choice(p.colptr[-1], size=64, replace=False)
    worst, worst_floor = 0.0, 0.0
    for e in ent:
        h = 1e-3 * max(abs(p.vals[e]), 1e-3)
        vp = vals0.clone(); vp[int(e)] += h
        vm = vals0.clone(); vm[int(e)] -= h
        fd = (loss(vp) - loss(vm)) / (2 * h)
        floor = 64 * np.finfo(float).eps * abs(l0) / h
        rel = abs(fd - Abar[e]) / abs(Abar[e])
        worst = max(worst, rel)
        worst_floor = max(worst_floor, floor / abs(Abar[e]))
        assert abs(fd - Abar[e]) <= 1e-5 * abs(Abar[e]) + floor, (int(e), fd, Abar[e])
    print(f"  FD on 64 entries: max rel error {worst:.2e} (largest rounding floor {worst_floor:.1e})", flush=True)
