"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the worked
example of Fig. 1 / Fig. 2, brute-force boolean elimination, closed-form
special patterns, LAPACK (numpy.linalg.cholesky), a planted factor L0,
closed-form grid-Laplacian eigenvalues, scipy's sparse LU and torch's dense
autograd.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import gen
import oracle


# --------------------------------------------------------------------------
# helpers (independent of the oracle)
# --------------------------------------------------------------------------

def csc_lower(M):
    """Lower triangle of a dense symmetric matrix (or pattern) as CSC arrays."""
    A = sp.csc_matrix(np.tril(M))
    A.sort_indices()
    return A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int64), A.data.astype(np.float64)


def brute_structure(pattern_lower_bool):
    """Boolean Gaussian elimination on a dense lower pattern: returns the
    filled lower pattern (numpy bool n x n)."""
    F = np.array(pattern_lower_bool, dtype=bool)
    n = F.shape[0]
    np.fill_diagonal(F, True)
    for k in range(n):
        below = [i for i in range(k + 1, n) if F[i, k]]
        for a in below:
            for b in below:
                if a > b:
                    F[a, b] = True
    return F


def permuted_pattern(n, colptr, rowind, perm):
    pinv = np.empty(n, np.int64)
    pinv[perm] = np.arange(n)
    P = np.zeros((n, n), bool)
    for j in range(n):
        for p in range(colptr[j], colptr[j + 1]):
            i = rowind[p]
            a, b = pinv[i], pinv[j]
            P[max(a, b), min(a, b)] = True
    return P


def random_pattern_problem(rng, n, density):
    n, cp, ri, vv = gen.random_spd(n, density, rng)
    perm = rng.permutation(n).astype(np.int64)
    return n, cp, ri, vv, perm


# --------------------------------------------------------------------------
# Fig. 1 / Fig. 2 worked example
# --------------------------------------------------------------------------

def _sn(label):
    return int(label[1:]) - 1


def test_fig1_maximal_supernodes(fig1_pattern, fig1_facts):
    n, cp, ri = fig1_pattern
    s = oracle.Symbolic(n, cp, ri, None, snode_mode=1, amalg_z=0)
    assert s.nnzL == cp[-1]  # the pattern is already a filled factor pattern
    expect = [[int(c) - 1 for c in f[1:]] for f in fig1_facts["supernode"]]
    got = [list(s.supernode_cols(J)) for J in range(s.nsuper)]
    assert got == expect
    for child, par in fig1_facts["sparent"]:
        assert s.sparent[_sn(child)] == _sn(par)
    assert s.sparent[5] == -1
    for lab, m, k in fig1_facts["storage"]:
        J = _sn(lab)
        assert len(s.supernode_rows(J)) == int(m)
        assert len(s.supernode_cols(J)) == int(k)


def test_fig1_updates_and_update_matrix(fig1_pattern, fig1_facts):
    n, cp, ri = fig1_pattern
    s = oracle.Symbolic(n, cp, ri, None, snode_mode=1, amalg_z=0)
    for f in fig1_facts["updates"]:
        J = _sn(f[0])
        targets = sorted(_sn(x) for x in f[1:])
        assert sorted(s.pair_P[s.pair_J == J].tolist()) == targets
    # Fig. 2: U_J1 is nonzero exactly at rows/cols {6, 7, 14}
    (lab, *rows), = fig1_facts["update_rows"]
    J = _sn(lab)
    k = len(s.supernode_cols(J))
    off = s.supernode_rows(J)[k:] + 1
    assert off.tolist() == [int(r) for r in rows]


def test_fig1_relind_positional(fig1_pattern, fig1_facts):
    n, cp, ri = fig1_pattern
    s = oracle.Symbolic(n, cp, ri, None, snode_mode=1, amalg_z=0)
    for J, P, *vals in fig1_facts["relind"]:
        assert s.relind(_sn(J), _sn(P)).tolist() == [int(v) for v in vals]
    # the printed [9, 8, 1] are 15 - i for the global rows i = 6, 7, 14
    (J, P, *printed), = fig1_facts["relind_printed"]
    J = _sn(J)
    k = len(s.supernode_cols(J))
    rows1 = s.supernode_rows(J)[k:] + 1
    assert [15 - i for i in rows1] == [int(v) for v in printed]


def test_fig1_rlb_blocks(fig1_pattern, fig1_facts):
    """RLB blocks (Sec. II-B): maximal runs of consecutive rows of J inside
    one ancestor supernode."""
    n, cp, ri = fig1_pattern
    s = oracle.Symbolic(n, cp, ri, None, snode_mode=1, amalg_z=0)
    (lab, *toks), = fig1_facts["blocks"]
    J = _sn(lab)
    k = len(s.supernode_cols(J))
    R = s.supernode_rows(J)[k:]
    owner = np.searchsorted(s.sptr, R, side="right") - 1
    blocks, cur = [], [R[0]]
    for a in range(1, len(R)):
        if R[a] == R[a - 1] + 1 and owner[a] == owner[a - 1]:
            cur.append(R[a])
        else:
            blocks.append(cur)
            cur = [R[a]]
    blocks.append(cur)
    expect = [[int(x) - 1 for x in blk.split()] for blk in " ".join(toks).split("|")]
    assert [list(map(int, b)) for b in blocks] == expect


def test_fig1_fundamental_partition(fig1_pattern):
    n, cp, ri = fig1_pattern
    s = oracle.Symbolic(n, cp, ri, None, snode_mode=0, amalg_z=0)
    # J3 = {5,6,7} and J6 = {12..15} are not fundamental: column 6 has the
    # etree children 2 and 5, column 13 has 9 and 12, column 14 has 7, 11, 13.
    assert (s.sptr + 1).tolist() == [1, 3, 5, 6, 8, 10, 12, 13, 14, 16]


# --------------------------------------------------------------------------
# structure vs brute force and closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_structure_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 41))
    n, cp, ri, vv, perm = random_pattern_problem(rng, n, rng.uniform(0.02, 0.3))
    s = oracle.Symbolic(n, cp, ri, perm, 0, 0)
    F = brute_structure(permuted_pattern(n, cp, ri, perm))
    for j in range(n):
        expect = np.nonzero(F[:, j])[0]
        assert s.lrow[s.lptr[j]:s.lptr[j + 1]].tolist() == expect.tolist()
        below = expect[expect > j]
        assert s.parent[j] == (below[0] if below.size else -1)
    # supernode row lists are the union of their columns' structures, and
    # (no amalgamation) every column of a supernode has the same rows below
    # the supernode's diagonal block
    for J in range(s.nsuper):
        cols = s.supernode_cols(J)
        rows = s.supernode_rows(J)
        union = np.nonzero(F[:, cols].any(axis=1))[0]
        assert rows.tolist() == union.tolist()
        last = cols[-1]
        for j in cols:
            assert np.nonzero(F[last + 1:, j])[0].tolist() == np.nonzero(F[last + 1:, last])[0].tolist()


def test_diagonal_pattern():
    n = 9
    s0 = oracle.Symbolic(n, np.arange(n + 1), np.arange(n), None, 0, 0)
    s1 = oracle.Symbolic(n, np.arange(n + 1), np.arange(n), None, 1, 0)
    assert s0.nsuper == n and s1.nsuper == n
    assert (s0.parent == -1).all()
    assert s0.npairs == 0


def test_tridiagonal_pattern():
    n = 12
    T = np.eye(n) * 4 - np.eye(n, k=-1) - np.eye(n, k=1)
    _, cp, ri, _ = csc_lower(T)
    s = oracle.Symbolic(n, cp, ri, None, 0, 0)
    assert s.parent.tolist() == list(range(1, n)) + [-1]
    assert s.sptr.tolist() == list(range(n - 1)) + [n]   # {0},...,{n-3},{n-2,n-1}


@pytest.mark.parametrize("z", [1, 2, 8])
def test_tridiagonal_amalgamation_closed_form(z):
    """Tridiagonal chain: the fundamental supernodes are {0}, ..., {n-3} and
    {n-2, n-1}.  A group of k columns ending before column n-2 has rows =
    its columns plus the next one: storage k(k+3)/2, 2k true nonzeros, so
    k(k-1)/2 explicit zeros.  A group of k columns ending at n-1 has storage
    k(k+1)/2, 2k - 1 true nonzeros and (k-1)(k-2)/2 zeros.  Merges are
    accepted while zeros <= z k."""
    n = 40
    T = np.eye(n) * 4 - np.eye(n, k=-1) - np.eye(n, k=1)
    _, cp, ri, _ = csc_lower(T)
    s = oracle.Symbolic(n, cp, ri, None, 0, z)
    expect, k, j = [0], 1, 0
    while True:
        if j + 1 == n - 2:          # the parent is the final pair
            kk = k + 2
            if (kk - 1) * (kk - 2) // 2 > z * kk:
                expect.append(n - 2)
            break
        kk = k + 1
        if kk * (kk - 1) // 2 <= z * kk:
            k = kk
        else:
            expect.append(j + 1)
            k = 1
        j += 1
    expect.append(n)
    assert s.sptr.tolist() == expect
    if z == 8:
        assert expect == [0, 17, 34, 40]


def test_arrowhead_pattern():
    n = 10
    M = np.eye(n) * n
    M[n - 1, :] = 1
    M[:, n - 1] = 1
    M[n - 1, n - 1] = n * n
    _, cp, ri, _ = csc_lower(M)
    s0 = oracle.Symbolic(n, cp, ri, None, 0, 0)
    s1 = oracle.Symbolic(n, cp, ri, None, 1, 0)
    assert s0.nsuper == n
    assert s1.sptr.tolist() == list(range(n - 1)) + [n]


def test_dense_pattern():
    n = 7
    M = np.ones((n, n)) + n * np.eye(n)
    _, cp, ri, _ = csc_lower(M)
    for mode in (0, 1):
        s = oracle.Symbolic(n, cp, ri, None, mode, 0)
        assert s.nsuper == 1 and s.sptr.tolist() == [0, n]
        assert s.flops() == sum((n - j) ** 2 for j in range(n))


@pytest.mark.parametrize("seed", range(6))
def test_amalgamation_properties(seed):
    """Every amalgamated supernode: columns contiguous, rows = union of its
    columns' true structures (brute force), explicit zeros <= z * k; the
    partition refines nothing it should not: merging only joins a supernode
    with the one right after it."""
    rng = np.random.default_rng(50 + seed)
    p = gen.make_config(0, seed=77 + seed, side=10)
    z = int(rng.integers(1, 9))
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
    base = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0)
    F = brute_structure(permuted_pattern(p.n, p.colptr, p.rowind, p.perm))
    counts = F.sum(axis=0)
    assert set(base.sptr.tolist()) >= set(s.sptr.tolist())
    for J in range(s.nsuper):
        cols = s.supernode_cols(J)
        rows = s.supernode_rows(J)
        assert rows.tolist() == np.nonzero(F[:, cols].any(axis=1))[0].tolist()
        k, m = len(cols), len(rows)
        storage = k * m - k * (k - 1) // 2
        assert storage - counts[cols].sum() <= z * k


def test_relind_definition_random():
    """relind(J,P)[t] = m_P - 1 - position of the row in P's row list, for
    J's off-diagonal rows from the first one inside P's columns."""
    p = gen.make_config(0, side=12)
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 4)
    owner = np.searchsorted(s.sptr, np.arange(p.n), side="right") - 1
    for t in range(s.npairs):
        J, P = s.pair_J[t], s.pair_P[t]
        k = s.sptr[J + 1] - s.sptr[J]
        R = s.supernode_rows(J)[k:]
        PR = list(s.supernode_rows(P))
        first = np.nonzero(owner[R] == P)[0][0]
        assert s.pair_a0[t] == first
        exp = [len(PR) - 1 - PR.index(i) for i in R[first:]]
        assert s.rel[s.relptr[t]:s.relptr[t + 1]].tolist() == exp


# --------------------------------------------------------------------------
# numeric
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_dense_vs_lapack(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 14))
    G = rng.standard_normal((n, n))
    M = G @ G.T + n * np.eye(n)
    n, cp, ri, vv = csc_lower(M)
    perm = rng.permutation(n)
    s = oracle.Symbolic(n, cp, ri, perm, 0, 0)
    for variant in (0, 1):
        f = s.factor(vv, variant)
        assert f.info == 0
        L = f.L_csc().toarray()
        Ld = np.linalg.cholesky(M[np.ix_(perm, perm)])
        np.testing.assert_allclose(L, Ld, rtol=0, atol=1e-12 * np.abs(Ld).max())


@pytest.mark.parametrize("seed", range(6))
def test_planted_factor(seed):
    """A = L0 L0^T on a filled (chordal) pattern => the factor is L0."""
    rng = np.random.default_rng(200 + seed)
    n = 30
    pat = np.tril(rng.random((n, n)) < 0.12, -1)
    F = brute_structure(pat)
    L0 = np.where(F, rng.uniform(-1, 1, (n, n)), 0.0)
    np.fill_diagonal(L0, rng.uniform(1.0, 2.0, n))
    A = L0 @ L0.T
    # store every position of the filled pattern (some may be exact zeros)
    Ls = sp.csc_matrix(np.where(F, A + 1e-300, 0.0))
    Ls.data -= 1e-300
    Ls.sort_indices()
    cp, ri = Ls.indptr.astype(np.int64), Ls.indices.astype(np.int64)
    vv = A[ri, np.repeat(np.arange(n), np.diff(cp))]
    s = oracle.Symbolic(n, cp, ri, None, 0, 0)
    for variant in (0, 1):
        f = s.factor(vv, variant)
        assert f.info == 0
        np.testing.assert_allclose(f.L_csc().toarray(), L0, atol=1e-12)


def test_residual_identity_cfg0():
    p = gen.make_config(0)
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0)
    f = s.factor(p.vals)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    Cm = A[p.perm][:, p.perm]
    L = f.L_csc()
    res = sp.linalg.norm(Cm - L @ L.T) / sp.linalg.norm(A)
    assert res <= 1e-15
    f1 = s.factor(p.vals, 1)
    np.testing.assert_allclose(f1.lv, f.lv, rtol=0, atol=1e-13 * np.abs(f.lv).max())


def _grid_logdet_closed_form(shape, shift):
    """Uniform-weight grid graph Laplacian + shift*I: eigenvalues are
    sum_d (2 - 2 cos(pi j_d / m_d)) + shift, j_d = 0..m_d-1 (Cartesian
    product of path graphs)."""
    lam = np.zeros(())
    for m in shape:
        ev = 2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m)
        lam = np.add.outer(lam, ev)
    return float(np.sum(np.log(lam.ravel() + shift)))


@pytest.mark.parametrize("shape,shift", [((32, 32), 1e-2), ((9, 7, 11), 1e-1), ((12, 12, 12), 1e-2)])
def test_logdet_closed_form(shape, shift):
    n, cp, ri, vv = gen.grid_laplacian(shape, None, "ones", shift=shift)
    perm = gen.nested_dissection(shape)
    s = oracle.Symbolic(n, cp, ri, perm, 0, 8)
    ld = s.factor(vv).logdet()
    assert abs(ld - _grid_logdet_closed_form(shape, shift)) <= 1e-11 * abs(ld)


@pytest.mark.parametrize("cfg", [0, 1, 2, 4])
def test_solve_vs_scipy(cfg):
    p = gen.make_config(cfg, side={0: 16, 1: 8, 2: 5, 4: 9}[cfg])
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, p.meta["amalg_z"])
    f = s.factor(p.vals)
    assert f.info == 0
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals).tocsc()
    X = f.solve(p.B)
    Xr = spla.spsolve(A, p.B)
    Xr = Xr.reshape(X.shape)
    np.testing.assert_allclose(X, Xr, rtol=1e-8, atol=1e-8 * np.abs(Xr).max())
    eta, _ = oracle.backward_error(A.tocsr(), X, p.B)
    assert eta.max() <= 1e-14


def test_not_spd_reports_first_column():
    # 2x2 indefinite: column 1 fine, column 2 pivot 1 - 4 < 0
    n, cp, ri, vv = csc_lower(np.array([[1.0, 2.0], [2.0, 1.0]]))
    s = oracle.Symbolic(n, cp, ri, None, 0, 0)
    assert s.factor(vv).info == 2 and s.factor(vv, 1).info == 2
    # diagonal with one negative entry at original index 5, permuted to 2
    n = 8
    d = np.ones(n)
    d[5] = -1.0
    perm = np.array([0, 1, 5, 2, 3, 4, 6, 7])
    s = oracle.Symbolic(n, np.arange(n + 1), np.arange(n), perm, 0, 0)
    assert s.factor(d).info == 3
    d[5] = np.nan
    assert s.factor(d).info == 3


def test_bad_inputs():
    with pytest.raises(oracle.OracleError):
        oracle.Symbolic(3, np.array([0, 1, 2, 3]), np.array([0, 1, 1]), None, 0, 0)  # upper entry
    with pytest.raises(oracle.OracleError):
        oracle.Symbolic(2, np.array([0, 1, 2]), np.array([0, 1]), np.array([0, 0]), 0, 0)  # bad perm
    with pytest.raises(oracle.OracleError):
        oracle.Symbolic(2, np.array([0, 1, 1]), np.array([1]), None, 0, 0)  # missing diagonal


def test_empty_and_one():
    s = oracle.Symbolic(0, np.array([0]), np.zeros(0, np.int64), None, 0, 0)
    assert s.nsuper == 0 and s.nnzL == 0
    s = oracle.Symbolic(1, np.array([0, 1]), np.array([0]), None, 0, 0)
    f = s.factor(np.array([4.0]))
    assert f.lv.tolist() == [2.0] and abs(f.logdet() - math.log(4.0)) < 1e-15


# --------------------------------------------------------------------------
# gradients vs torch dense autograd
# --------------------------------------------------------------------------

def test_gradients_vs_torch_dense():
    torch = pytest.importorskip("torch")
    p = gen.make_config(0, side=5)
    n = p.n
    s = oracle.Symbolic(n, p.colptr, p.rowind, p.perm, 0, 0)
    f = s.factor(p.vals)
    b = p.B[:, 0]
    x = f.solve(b)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(n)
    g_ld = oracle.grad_logdet(f, p.colptr, p.rowind)
    g_x, lam = oracle.grad_solve(f, p.colptr, p.rowind, x, c)

    r, col = oracle.entry_coords(p.colptr, p.rowind)
    v = torch.tensor(p.vals, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
    A = torch.zeros((n, n), dtype=torch.float64)
    A = A.index_put((torch.tensor(r), torch.tensor(col)), v)
    A = A + A.T - torch.diag(torch.diagonal(A))
    ld = torch.logdet(A)
    (gv,) = torch.autograd.grad(ld, v, retain_graph=True)
    np.testing.assert_allclose(g_ld, gv.numpy(), rtol=1e-10, atol=1e-12)
    xt = torch.linalg.solve(A, bt)
    loss = (xt * torch.tensor(c)).sum()
    gv2, gb = torch.autograd.grad(loss, (v, bt))
    np.testing.assert_allclose(g_x, gv2.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(lam.ravel(), gb.numpy(), rtol=1e-9, atol=1e-12)


def test_backward_error_hand_example():
    A = sp.csr_matrix(np.array([[2.0, -1.0], [-1.0, 2.0]]))
    x = np.array([1.0, 1.0])
    b = np.array([1.0, 2.0])
    # r = b - A x = [0, 1]; ||A||_inf = 3; eta = 1 / (3*1 + 2)
    eta, comp = oracle.backward_error(A, x, b)
    assert abs(eta[0] - 0.2) < 1e-16
    # |A||x| + |b| = [3+1, 3+2]; componentwise max(0/4, 1/5)
    assert abs(comp[0] - 0.2) < 1e-16


def test_prefix_columns_equal_full_factor():
    """Column j of L depends only on columns k < j: a factorization stopped
    after t columns agrees with the full one on those columns, bit for bit."""
    p = gen.make_config(4, side=10)
    s = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    full = s.factor(p.vals)
    t = p.n // 3
    part = s.factor(p.vals, ncols=t)
    e = s.lptr[t]
    assert np.array_equal(part.lv[:e], full.lv[:e])
    assert not part.lv[e:].any()
    assert s.flops(t) == float((s.count[:t].astype(np.float64) ** 2).sum())
    with pytest.raises(oracle.OracleError):
        part.solve(p.B)
