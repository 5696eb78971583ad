"""Input generators: shapes, symmetry, definiteness, orderings."""
import numpy as np
import pytest

import gen


def full(p_or_tuple):
    n, cp, ri, vv = p_or_tuple
    return gen.full_from_lower(n, cp, ri, vv)


@pytest.mark.parametrize("shape", [(5, 4), (4, 3, 5), (32, 32)])
def test_nested_dissection_is_permutation(shape):
    perm = gen.nested_dissection(shape)
    assert sorted(perm.tolist()) == list(range(int(np.prod(shape))))


def test_nested_dissection_top_separator_last():
    perm = gen.nested_dissection((7, 5))
    # longest axis x (extent 7): mid = 3, separator = the column x == 3
    last = perm[-5:]
    assert sorted((last % 7).tolist()) == [3] * 5
    # lexicographic, x fastest: y ascending
    assert (last // 7).tolist() == [0, 1, 2, 3, 4]


def test_laplacian_row_sums_equal_shift():
    rng = np.random.default_rng(0)
    A = full(gen.grid_laplacian((6, 5, 4), rng, "loguniform", -2, 2, shift=1e-3))
    np.testing.assert_allclose(np.asarray(A.sum(axis=1)).ravel(), 1e-3, atol=1e-9)
    assert (A - A.T).nnz == 0


def test_config0_shape_and_spd():
    p = gen.make_config(0)
    assert p.n == 1024 and p.B.shape == (1024, 1)
    A = full((p.n, p.colptr, p.rowind, p.vals)).toarray()
    w = np.linalg.eigvalsh(A)
    assert w.min() > 0.009  # shift 1e-2 on a PSD Laplacian
    off = -A[np.tril_indices(p.n, -1)]
    off = off[off != 0]
    assert off.min() >= 0.5 and off.max() <= 1.5


def test_elasticity_blocks_spd():
    rng = np.random.default_rng(1)
    n, cp, ri, vv = gen.elasticity_27pt(3, rng)
    A = full((n, cp, ri, vv)).toarray()
    assert n == 81
    np.testing.assert_allclose(A, A.T)
    w = np.linalg.eigvalsh(A)
    assert w.min() >= 1e-2 - 1e-9
    # an off-diagonal block is -K with eigenvalues in [1, 10]
    K = -A[3:6, 0:3]
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev.min() >= 1 - 1e-9 and ev.max() <= 10 + 1e-9


def test_grf_normalised():
    rng = np.random.default_rng(2)
    g = gen.gaussian_random_field((16, 16, 16), rng, ell=4.0)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12


def test_batch_plan():
    probs = gen.make_batch(count=16, nrhs=4)
    for p in probs:
        s = p.meta["shape"]
        if len(s) == 2:
            assert 12 <= s[0] <= 48
        else:
            assert 8 <= s[0] <= 20
        assert p.B.shape == (p.n, 4)


def test_seeds_deterministic():
    a = gen.make_config(0)
    b = gen.make_config(0)
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.B, b.B)
