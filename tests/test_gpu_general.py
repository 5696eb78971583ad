"""General-pattern path on the GPU: patterns ordered by the library's own
nested dissection and merged by the greedy rule of Sec. IV-A (25 % cap),
factored, solved and reduced to logdet, against the oracle on the same
ordering and structure.  Gates as for the grid workloads: the factor is
unique, so L on the oracle's structure within 1e-12 relative (Frobenius),
backward error <= 1e-12, logdet within 1e-12 relative."""
import numpy as np
import pytest

import gen
import oracle
from conftest import gpu_available
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

torch = pytest.importorskip("torch")
sc = pytest.importorskip("paper_2409_14009_amd")


def _random_geometric(n, k, seed):
    """SPD matrix on a random geometric graph in the unit cube (each point
    joined to its k nearest neighbours; no grid structure), weights
    U[0.5, 1.5], diagonal = row sum + 1e-2."""
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    X = rng.random((n, 3))
    _, nb = cKDTree(X).query(X, k + 1)
    i = np.repeat(np.arange(n), k)
    j = nb[:, 1:].ravel()
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo * n + hi)
    lo, hi = key // n, key % n
    w = rng.uniform(0.5, 1.5, size=lo.size)
    W = sp.coo_matrix((w, (hi, lo)), shape=(n, n)).tocsc()
    d = np.asarray((W + W.T).sum(axis=1)).ravel() + 1e-2
    Lw = (-W + sp.diags(d)).tocsc()
    Lw = sp.tril(Lw).tocsc()
    Lw.sort_indices()
    return n, Lw.indptr.astype(np.int64), Lw.indices.astype(np.int64), Lw.data.copy(), rng.standard_normal((n, 2))


CASES = {
    "geometric_6000_k8": lambda: _random_geometric(6000, 8, 1),
    "random_spd_1500": lambda: (lambda r: (lambda t: t + (r.standard_normal((t[0], 2)),))(
        gen.random_spd(1500, 0.004, r)))(np.random.default_rng(2)),
    "elasticity_8": lambda: (lambda p: (p.n, p.colptr, p.rowind, p.vals, p.B))(gen.make_config(2, side=8)),
    "grf_20": lambda: (lambda p: (p.n, p.colptr, p.rowind, p.vals, p.B))(gen.make_config(4, side=20)),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("cap", [25])
def test_nd_greedy_factor_solve_logdet(name, cap):
    n, cp, ri, vv, B = CASES[name]()
    perm = sc.order_nd(n, cp, ri)
    S = sc.SparseCholesky(n, cp, ri, perm, 0, 0, amalg_rule=1, amalg_cap_percent=cap)
    inf = S.info()
    print(f"general case {name}: n={n} nsuper={inf['nsuper']} nnz_l={inf['nnz_l']} storage={inf['storage']}",
          flush=True)
    F = S.factor(torch.tensor(vv, device="cuda"))
    X = F.solve(torch.tensor(B, device="cuda")).cpu().numpy()
    Lst = F.storage().cpu().numpy()
    ld = F.logdet()
    of = oracle.Symbolic(n, cp, ri, perm, 0, 0, amalg_rule=1, amalg_cap_percent=cap).factor(vv)
    assert of.info == 0
    A = oracle.full_matrix(n, cp, ri, vv)
    Cm = permuted_matrix(A, perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), Lst, n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    eta, _ = oracle.backward_error(A, X, B)
    rel_ld = abs(ld - of.logdet()) / abs(of.logdet())
    print(f"  frobenius {fro:.2e} elementwise {elt:.2e} eta {eta.max():.2e} logdet {rel_ld:.2e}", flush=True)
    assert upper == 0.0 and offmax == 0.0
    assert fro <= 1e-12 and eta.max() <= 1e-12 and rel_ld <= 1e-12
