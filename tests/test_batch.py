"""Batched analysis (block-diagonal union of independent matrices): the
structure of every block equals that matrix's own structure (CPU)."""
import numpy as np
import pytest

import gen
import oracle

sc = pytest.importorskip("paper_2409_14009_amd")


@pytest.mark.parametrize("z", [0, 8])
def test_batch_structure_matches_each_matrix(z):
    probs = gen.make_batch(count=12, nrhs=2)
    mats = [(p.n, p.colptr, p.rowind, p.perm) for p in probs]
    B = sc.BatchCholesky(mats, amalg_max_zeros=z)
    cnt, co, no = B.batch_info()
    assert cnt == 12
    assert np.array_equal(np.diff(co), [p.n for p in probs])
    assert np.array_equal(np.diff(no), [p.nnz for p in probs])
    e = B.export()
    inf = B.info()
    tot_flops = 0.0
    sp_ = e["super_ptr"]
    for b, p in enumerate(probs):
        o = oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z)
        tot_flops += o.flops()
        # supernodes of block b
        sel = (sp_[:-1] >= co[b]) & (sp_[:-1] < co[b + 1])
        idx = np.nonzero(sel)[0]
        assert np.array_equal(sp_[idx] - co[b], o.sptr[:-1])
        for t, J in enumerate(idx):
            rows = e["row_idx"][e["row_ptr"][J]:e["row_ptr"][J + 1]] - co[b]
            assert np.array_equal(rows, o.supernode_rows(t))
            par = e["sparent"][J]
            assert (par - idx[0] if par >= 0 else -1) == o.sparent[t]
        # parent of the block's columns stays inside the block
        par = e["parent"][co[b]:co[b + 1]]
        assert np.all((par == -1) | ((par >= co[b]) & (par < co[b + 1])))
    assert inf["flops_alg"] == tot_flops
    assert inf["nsuper"] == sum(oracle.Symbolic(p.n, p.colptr, p.rowind, p.perm, 0, z).nsuper for p in probs)


def test_batch_arguments():
    with pytest.raises(sc.SpcholError):
        sc.BatchCholesky([(3, np.array([0, 1, 2, 3]), np.array([0, 1, 2]), np.array([0, 0, 1]))])
    S = sc.BatchCholesky([])
    assert S.batch_info()[0] == 0 and S.info()["n"] == 0
