"""General-pattern symbolic analysis (host, no GPU): the library's own
nested-dissection ordering (a stand-in for the METIS ordering of Sec. IV-A)
and the greedy supernode merging of Sec. IV-A (least new fill first, up to
a cap on the storage increase).

Pins of the greedy rule on the oracle side (independent of the library):
a closed form for the path graph, the cap-0 case equal to the maximal
supernode partition (a merge adds no fill exactly when the two column
structures nest), and the cap itself.  The library's analysis is then
compared with the oracle bit-exactly.  The ordering is checked for being a
permutation, for its fill against the geometric dissection of the grid
workloads, and for the separator property of its top split.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle

sc = pytest.importorskip("paper_2409_14009_amd")


def _path(n):
    cp, ri = [0], []
    for j in range(n):
        ri.append(j)
        if j + 1 < n:
            ri.append(j + 1)
        cp.append(len(ri))
    return n, np.array(cp, np.int64), np.array(ri, np.int64)


def _trap(k, m):
    return k * m - k * (k - 1) // 2


# --- oracle pins of the greedy rule ----------------------------------------

@pytest.mark.parametrize("n,expect", [
    # cap 9: the nine pairs {0,1} .. {16,17}; {18,19} was fundamental already
    (20, list(range(0, 21, 2))),
    # cap 10: nine pairs, then {18} into {19,20} (one zero: rows 18..20)
    (21, list(range(0, 19, 2)) + [21]),
    # cap 19: the nineteen pairs {0,1} .. {36,37}
    (40, list(range(0, 41, 2))),
])
def test_oracle_greedy_path_closed_form(n, expect):
    """Path graph, natural order: fundamental supernodes {0}, ..., {n-3},
    {n-2, n-1}.  Merging a singleton into a singleton parent, or into the
    last two-column supernode, adds one explicit zero; merging a two-column
    group into a singleton adds two.  Least fill first, ties to the smaller
    first column, gives the pairs {0,1}, {2,3}, ... until the cap, 25 % of
    nnz(L) = 2n - 1 (integer part), is spent."""
    n, cp, ri = _path(n)
    o = oracle.Symbolic(n, cp, ri, None, 0, 0, amalg_rule=1, amalg_cap_percent=25)
    assert o.sptr.tolist() == expect


@pytest.mark.parametrize("seed", range(8))
def test_oracle_greedy_cap0_is_maximal(seed):
    """With no fill allowed only pairs whose structures nest merge, which is
    the maximal supernode partition."""
    rng = np.random.default_rng(100 + seed)
    n, cp, ri, _ = gen.random_spd(int(rng.integers(30, 160)), rng.uniform(0.01, 0.1), rng)
    perm = rng.permutation(n)
    g = oracle.Symbolic(n, cp, ri, perm, 0, 0, amalg_rule=1, amalg_cap_percent=0)
    mx = oracle.Symbolic(n, cp, ri, perm, 1, 0)
    assert np.array_equal(g.sptr, mx.sptr)
    assert np.array_equal(g.srow, mx.srow)


@pytest.mark.parametrize("cap", [5, 25, 80])
def test_oracle_greedy_respects_cap_and_merges(cap):
    p = gen.make_config(1, side=8)
    base = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0)
    g = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, 0, amalg_rule=1, amalg_cap_percent=cap)
    store = sum(_trap(int(g.sptr[J + 1] - g.sptr[J]), int(g.srptr[J + 1] - g.srptr[J])) for J in range(g.nsuper))
    assert store - g.nnzL <= g.nnzL * cap // 100
    assert g.nsuper < base.nsuper
    # every supernode is a run of whole fundamental supernodes
    assert set(g.sptr.tolist()) <= set(base.sptr.tolist())


# --- the library's analysis against the oracle -------------------------------

def _structure_equal(n, cp, ri, perm, mode, cap):
    S = sc.SparseCholesky(n, cp, ri, perm, mode, 0, amalg_rule=1, amalg_cap_percent=cap)
    e = S.export()
    o = oracle.Symbolic(n, cp, ri, perm, mode, 0, amalg_rule=1, amalg_cap_percent=cap)
    for k, ok in (("super_ptr", o.sptr), ("sparent", o.sparent), ("row_ptr", o.srptr), ("row_idx", o.srow),
                  ("pair_J", o.pair_J), ("pair_P", o.pair_P), ("relind_ptr", o.relptr), ("relind", o.rel)):
        assert np.array_equal(e[k], ok), k
    return S


@pytest.mark.parametrize("cfg,side", [(0, 32), (1, 10), (2, 5), (4, 12)])
@pytest.mark.parametrize("cap", [0, 10, 25, 60])
def test_greedy_structure_bit_exact(cfg, side, cap):
    p = gen.make_config(cfg, side=side)
    perm = sc.order_nd(p.n, p.colptr, p.rowind)
    _structure_equal(p.n, p.colptr, p.rowind, perm, 0, cap)


@pytest.mark.parametrize("seed", range(6))
def test_greedy_structure_random_patterns(seed):
    rng = np.random.default_rng(seed)
    n, cp, ri, _ = gen.random_spd(int(rng.integers(20, 220)), rng.uniform(0.01, 0.1), rng)
    _structure_equal(n, cp, ri, rng.permutation(n), int(rng.integers(0, 2)), int(rng.integers(0, 50)))


# --- the ordering --------------------------------------------------------------

def test_order_nd_permutation_and_determinism():
    p = gen.make_config(1, side=12)
    a = sc.order_nd(p.n, p.colptr, p.rowind, 64, 7)
    b = sc.order_nd(p.n, p.colptr, p.rowind, 64, 7)
    assert np.array_equal(np.sort(a), np.arange(p.n))
    assert np.array_equal(a, b)
    # the full symmetric pattern gives the same ordering as the lower one
    Lw = sp.csc_matrix((np.ones(len(p.rowind)), p.rowind, p.colptr), shape=(p.n, p.n))
    F = (Lw + Lw.T).tocsc()
    F.sort_indices()
    c = sc.order_nd(p.n, F.indptr.astype(np.int64), F.indices.astype(np.int64), 64, 7)
    assert np.array_equal(a, c)


def test_order_nd_edge_cases():
    assert sc.order_nd(0, np.array([0]), np.zeros(0, np.int64)).size == 0
    assert sc.order_nd(1, np.array([0, 1]), np.array([0])).tolist() == [0]
    # two disconnected paths: a permutation, both components kept apart
    n, cp, ri = _path(300)
    ri2 = ri.copy()
    keep = ~((ri == 150) & (np.repeat(np.arange(n), np.diff(cp)) == 149))
    cols = np.repeat(np.arange(n), np.diff(cp))[keep]
    M = sp.csc_matrix((np.ones(keep.sum()), (ri2[keep], cols)), shape=(n, n))
    M.sort_indices()
    perm = sc.order_nd(n, M.indptr.astype(np.int64), M.indices.astype(np.int64), 16)
    assert np.array_equal(np.sort(perm), np.arange(n))
    with pytest.raises(sc.SpcholError):
        sc.order_nd(2, np.array([0, 1, 2]), np.array([0, 5]))


@pytest.mark.parametrize("cfg,side,bound", [(0, 32, 1.10), (1, 16, 1.10), (1, 24, 1.10), (4, 16, 1.10), (2, 8, 1.35)])
def test_order_nd_fill_against_geometric(cfg, side, bound):
    """The grid workloads come with a geometric nested dissection (the
    separator planes); the graph-only ordering must reach about the same
    fill, far below the natural order's."""
    p = gen.make_config(cfg, side=side)
    perm = sc.order_nd(p.n, p.colptr, p.rowind)
    geo = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm).info()["nnz_l"]
    ours = sc.SparseCholesky(p.n, p.colptr, p.rowind, perm).info()["nnz_l"]
    nat = sc.SparseCholesky(p.n, p.colptr, p.rowind, None).info()["nnz_l"]
    print(f"cfg {cfg} side {side}: nnz(L) geometric {geo} ours {ours} ({ours / geo:.3f}) natural {nat}")
    assert ours <= bound * geo
    assert ours < 0.8 * nat


def test_order_nd_top_separator_2d():
    """2D 5-point grid: the last-eliminated block is a separator of about one
    grid line, and removing it disconnects the rest."""
    side = 40
    p = gen.make_config(0, side=side)
    perm = sc.order_nd(p.n, p.colptr, p.rowind)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, perm)
    e = S.export()
    root = int(np.argmax(e["level"]))
    k = int(e["super_ptr"][root + 1] - e["super_ptr"][root])
    assert side <= k <= 1.3 * side
    sep = set(perm[e["super_ptr"][root]:e["super_ptr"][root + 1]].tolist())
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, np.ones(len(p.rowind))).tolil()
    rest = [v for v in range(p.n) if v not in sep]
    sub = sp.csr_matrix(A)[rest][:, rest]
    ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
    assert ncomp >= 2
