"""Host-resident factorization with every supernode below the size
threshold: no device call at all, so it runs here.  The factor is unique:
compared with the oracle's entry by entry; the host work is parallel over
update columns with distinct targets, so the result is the same bits for
any thread count; a non-positive pivot is reported like spchol_factor."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import compare_factor, permuted_matrix, storage_to_csc

sc = pytest.importorskip("paper_2409_14009_amd")

HOST_ONLY = 1 << 62


@pytest.mark.parametrize("cfg,side,z", [(0, 32, 0), (2, 6, 8), (4, 14, 8), (1, 10, 0)])
def test_host_only_factor_vs_oracle(cfg, side, z):
    p = gen.make_config(cfg, side=side)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, z)
    L, info, st = S.factor_streamed(p.vals, host_threshold=HOST_ONLY)
    assert info == 0 and st["gpu_supernodes"] == 0 and st["device_bytes"] == 0
    assert st["host_supernodes"] == S.info()["nsuper"]
    of = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z).factor(p.vals)
    A = oracle.full_matrix(p.n, p.colptr, p.rowind, p.vals)
    Cm = permuted_matrix(A, p.perm)
    Lg, upper = storage_to_csc(S.export(), S.storage_offsets(), L, p.n)
    elt, offmax, fro = compare_factor(Lg, of.L_csc(), Cm.diagonal())
    assert upper == 0.0 and offmax == 0.0 and fro <= 1e-12 and elt <= 1e-10
    # the same bits with one thread
    L1, _, st1 = S.factor_streamed(p.vals, host_threshold=HOST_ONLY, host_threads=1)
    assert st1["host_threads"] == 1
    assert np.array_equal(L.view(np.uint64), L1.view(np.uint64))


def test_host_only_not_spd():
    p = gen.make_config(0, side=12)
    v = p.vals.copy()
    v[p.colptr[40]] = -1.0  # diagonal entry of original column 40
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm)
    with pytest.raises(sc.NotPositiveDefinite) as ei:
        S.factor_streamed(v, host_threshold=HOST_ONLY)
    o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm).factor(v)
    assert ei.value.info == o.info > 0
