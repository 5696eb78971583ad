"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Gates (from the fp64 arithmetic and the workloads' stated tolerances):
  * structure: bit-exact (tests/test_capi.py, CPU);
  * factor: relative residual ||C - L L^T||_F / ||C||_F <= 1e-12, and where
    the matrix is well conditioned (kappa <~ 1e4: the 2D configuration and the
    diagonally dominant random matrices) ||L - L_oracle||_F / ||L_oracle||_F
    <= 1e-12 and |L_ij - Lo_ij| <= 1e-12 sqrt(C_ii) entry by entry (|L_ij| <=
    sqrt(C_ii) bounds every entry of row i);
  * explicit zeros of amalgamation are exactly 0 (they only ever receive
    products with an exact zero factor);
  * solve: normwise backward error <= 1e-12;
  * logdet: relative difference to the oracle <= 1e-12.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, residual_rel, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")

DEV = "cuda"


def _announce(msg):
    print(msg, flush=True)


def run_case(n, cp, ri, vv, perm, B, mode=0, z=0, nb=64, well_conditioned=True, check_L=True):
    _announce(f"case n={n} mode={mode} z={z} nb={nb}")
    S = sc.SparseCholesky(n, cp, ri, perm, mode, z, nb)
    F = S.factor(torch.tensor(vv, device=DEV))
    X = F.solve(torch.tensor(B, device=DEV)).cpu().numpy()
    ld = F.logdet()
    Lst = F.storage().cpu().numpy()
    torch.cuda.synchronize()
    osym = oracle.Symbolic(n, cp, ri, perm, mode, z)
    ofac = osym.factor(vv)
    assert ofac.info == 0
    A = oracle.full_matrix(n, cp, ri, vv)
    res = {}
    if check_L:
        Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), Lst, n)
        assert upper == 0.0
        Cm = permuted_matrix(A, osym.perm if perm is not None else np.arange(n))
        elt, offmax, fro = compare_factor(Lg, ofac.L_csc(), Cm.diagonal())
        assert offmax == 0.0, "explicit zeros must stay exactly zero"
        r = residual_rel(Cm, Lg)
        res.update(elt=elt, fro=fro, resid=r)
        assert r <= 1e-12, r
        if well_conditioned:
            assert fro <= 1e-12, fro
            assert elt <= 1e-12, elt
    eta, _ = oracle.backward_error(A, X, B)
    res["eta"] = float(eta.max())
    assert eta.max() <= 1e-12, eta
    ldo = ofac.logdet()
    res["logdet"] = abs(ld - ldo) / max(abs(ldo), 1.0)
    assert res["logdet"] <= 1e-12, (ld, ldo)
    if well_conditioned:
        Xo = ofac.solve(B)
        ex = np.abs(X - Xo).max() / np.abs(Xo).max()
        res["x"] = ex
        assert ex <= 1e-10, ex
    _announce(f"  ok {res}")
    return S, F


def test_config0_fundamental():
    p = gen.make_config(0)
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, p.B, 0, 0)


@pytest.mark.parametrize("mode,z,nb", [(1, 0, 64), (0, 8, 64), (0, 8, 16), (0, 3, 32), (1, 8, 48)])
def test_config0_variants(mode, z, nb):
    p = gen.make_config(0)
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, p.B, mode, z, nb)


@pytest.mark.parametrize("seed", range(8))
def test_random_spd(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 400))
    n, cp, ri, vv = gen.random_spd(n, rng.uniform(0.005, 0.08), rng)
    perm = rng.permutation(n)
    B = rng.standard_normal((n, int(rng.integers(1, 9))))
    run_case(n, cp, ri, vv, perm, B, int(rng.integers(0, 2)), int(rng.integers(0, 12)),
             int(rng.choice([16, 32, 48, 64])))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 200])
def test_dense(n):
    """One supernode: panels, ragged last panel, internal updates."""
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n))
    M = G @ G.T / n + np.eye(n)
    Ls = sp.csc_matrix(np.tril(M))
    Ls.sort_indices()
    B = rng.standard_normal((n, 3))
    run_case(n, Ls.indptr.astype(np.int64), Ls.indices.astype(np.int64), Ls.data, rng.permutation(n), B,
             0, 0, 64)


@pytest.mark.parametrize("n,nb", [(150, 64), (150, 32), (300, 48), (333, 64), (400, 64), (1000, 64)])
def test_dense_odd_panels(n, nb):
    """One dense supernode (odd panel counts and a ragged last panel among
    the cases), several blocks of right-hand sides; with 64-column panels and six, seven or 16
    of them, several one-launch panel rounds with trailing update tiles
    (at 16, column blocks entering the rounds' window with all their
    finished panels at once)."""
    rng = np.random.default_rng(n + nb)
    G = rng.standard_normal((n, n))
    M = G @ G.T / n + np.eye(n)
    Ls = sp.csc_matrix(np.tril(M))
    Ls.sort_indices()
    B = rng.standard_normal((n, 5))
    run_case(n, Ls.indptr.astype(np.int64), Ls.indices.astype(np.int64), Ls.data, rng.permutation(n), B,
             0, 0, nb)


@pytest.mark.parametrize("side,nb,nrhs", [(14, 16, 1), (16, 48, 6), (14, 32, 9)])
def test_backward_split_rounds(side, nb, nrhs):
    """Separators of many panels with hundreds of rows below them: backward
    panels split into far row tiles a round ahead and a finishing task,
    several blocks of four right-hand sides."""
    p = gen.make_config(2, side=side)
    B = np.random.default_rng(side * nb + nrhs).standard_normal((p.n, nrhs))
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, B, 0, 8, nb)


@pytest.mark.parametrize("cfg,side", [(1, 16), (2, 7), (4, 16)])
def test_reduced_configs(cfg, side):
    """The 3D recipes on smaller grids: multi-panel separators, amalgamation."""
    p = gen.make_config(cfg, side=side)
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, p.B, 0, 8, 64, well_conditioned=(cfg != 1))


def test_not_spd_reports_column():
    p = gen.make_config(0, side=12)
    vv = p.vals.copy()
    # make one diagonal entry negative enough to break definiteness
    diag_pos = p.colptr[:-1]
    vv[diag_pos[70]] = -5.0
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 0)
    with pytest.raises(sc.NotPositiveDefinite) as ei:
        S.factor(torch.tensor(vv, device=DEV))
    o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0).factor(vv)
    assert ei.value.info == o.info > 0
    F = S.factor(torch.tensor(vv, device=DEV), check=False)
    assert F.info == o.info
    # NaN input
    vv[diag_pos[3]] = np.nan
    F = S.factor(torch.tensor(vv, device=DEV), check=False)
    o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0).factor(vv)
    assert F.info == o.info > 0


def test_refactor_and_raw_ldb():
    p = gen.make_config(4, side=10)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    F = S.factor(torch.tensor(p.vals, device=DEV))
    v2 = p.vals * 1.5
    F.refactor(torch.tensor(v2, device=DEV))
    o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8).factor(v2)
    assert abs(F.logdet() - o.logdet()) <= 1e-12 * abs(o.logdet())
    # raw ABI with a leading dimension larger than n
    nrhs, ldb = 3, p.n + 7
    rng = np.random.default_rng(0)
    Bh = rng.standard_normal((nrhs, ldb))
    Bd = torch.tensor(Bh, device=DEV)
    st = torch.cuda.current_stream().cuda_stream
    rc = sc.lib().spchol_solve(F._h, C.c_void_p(Bd.data_ptr()), nrhs, ldb, C.c_void_p(st))
    assert rc == 0
    Xh = Bd.cpu().numpy()
    Xo = o.solve(Bh[:, :p.n].T.copy())
    np.testing.assert_allclose(Xh[:, :p.n].T, Xo, rtol=1e-9, atol=1e-12)
    assert np.array_equal(Xh[:, p.n:], Bh[:, p.n:])  # padding untouched
    assert sc.lib().spchol_solve(F._h, C.c_void_p(Bd.data_ptr()), nrhs, p.n - 1, C.c_void_p(st)) == -1


def test_empty_and_one():
    S = sc.SparseCholesky(1, np.array([0, 1]), np.array([0]))
    F = S.factor(torch.tensor([9.0], device=DEV, dtype=torch.float64))
    x = F.solve(torch.tensor([3.0], device=DEV, dtype=torch.float64))
    assert abs(float(x[0]) - 1.0 / 3.0) < 1e-16
    assert abs(F.logdet() - np.log(9.0)) < 1e-15
    S0 = sc.SparseCholesky(0, np.array([0]), np.zeros(0, np.int64))
    F0 = S0.factor(torch.zeros(0, device=DEV, dtype=torch.float64))
    assert F0.logdet() == 0.0


def test_wide_supernodes_big_tiles():
    """18^3 7-point grid: separators of >= 128 columns that still update
    their ancestors (several panels feeding multi-tile external updates)."""
    p = gen.make_config(1, side=18)
    e = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8).export()
    k = np.diff(e["super_ptr"]); m = np.diff(e["row_ptr"])
    assert ((k >= 128) & (m > k)).any()
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, p.B, 0, 8, 64, well_conditioned=False)


@pytest.mark.parametrize("k,r", [(1, 59), (4, 56), (4, 57), (5, 43), (16, 32), (16, 33), (17, 10), (3, 0),
                                 (16, 0), (8, 1)])
def test_small_supernode_limits(k, r):
    """Leaves at and past the limits of the one-wavefront supernode (two
    leaves of k columns updating a parent of r rows): the same factor,
    solve and log-determinant either way."""
    rng = np.random.default_rng(2000 * k + r)
    n, cp, ri, vv = gen.leaf_pair_spd(k, r, rng)
    B = rng.standard_normal((n, 3))
    run_case(n, cp, ri, vv, None, B, 0, 0, 64)


@pytest.mark.parametrize("k,r", [(1, 60), (4, 57), (16, 33), (16, 160), (7, 150), (12, 129), (16, 161), (17, 40),
                                 (20, 5), (32, 0), (32, 100), (24, 160), (33, 50)])
def test_medium_supernodes(k, r):
    """Short one-panel leaves of at most 32 columns not done by the
    whole-step one-wavefront task: factored one wavefront each (the rows
    below past the sweep in 64-row chunks), their update by the external
    tiles; (16, 161) and (33, 50) just past the limits."""
    print(f"case medium leaves k={k} r={r}", flush=True)
    rng = np.random.default_rng(4000 * k + r)
    n, cp, ri, vv = gen.leaf_pair_spd(k, r, rng)
    B = rng.standard_normal((n, 3))
    run_case(n, cp, ri, vv, None, B, 0, 0, 64)


@pytest.mark.parametrize("cfg,side,z,nrhs", [(4, 16, 8, 1), (4, 16, 8, 3), (4, 16, 8, 4), (4, 16, 8, 6),
                                             (0, None, 0, 5), (2, 14, 8, 8)])
def test_small_solve_levels(cfg, side, z, nrhs):
    """Leaf levels with >= 256 supernodes of one small panel (<= 16
    columns, <= 128 rows below) are solved one wavefront each, for several
    right-hand-side counts, beside levels just under the threshold that
    keep the ordinary rounds."""
    p = gen.make_config(cfg, side=side) if side else gen.make_config(cfg)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    e = S.export()
    k = np.diff(e["super_ptr"]); m = np.diff(e["row_ptr"]); lev = e["level"]
    q = (k <= 16) & (m - k <= 128)
    per_level = [int((q & (lev == l)).sum()) for l in range(int(lev.max()) + 1)]
    assert max(per_level) >= 256 and any(0 < c < 256 for c in per_level), per_level
    if cfg == 2:
        # leaves of 3-dof points: 65..128 rows below (two rows a lane)
        big = q & (m - k > 64) & (lev == int(np.argmax(per_level)))
        assert big.sum() > 0
    B = np.random.default_rng(77 + nrhs).standard_normal((p.n, nrhs))
    run_case(p.n, p.colptr, p.rowind, p.vals, p.perm, B, 0, z, 64)
