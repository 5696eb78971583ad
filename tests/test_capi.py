"""C ABI: symbols, argument checking and the host-side analysis (no GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import gen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

sc = pytest.importorskip("paper_2409_14009_amd")


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(spchol_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = sc.lib()
    names = _declared_functions()
    assert len(names) >= 12
    for name in sorted(names):
        assert hasattr(lib, name), name
    # and the binding declares a prototype for each
    from paper_2409_14009_amd import _capi
    assert names <= set(_capi.PROTOTYPES)


def test_version_and_defaults():
    assert "spchol" in sc.version()
    from paper_2409_14009_amd import _capi
    o = _capi.Options()
    assert sc.lib().spchol_default_options(C.byref(o)) == 0
    assert (o.snode_mode, o.amalg_max_zeros, o.panel_width, o.deterministic, o.workspace_limit) == (0, 0, 64, 0, 0)


def _status(n, cp, ri, perm=None, opts=None):
    h = C.c_void_p()
    ptr = lambda a: None if a is None else np.ascontiguousarray(a, np.int64).ctypes.data_as(C.c_void_p)
    keep = [np.ascontiguousarray(a, np.int64) if a is not None else None for a in (cp, ri, perm)]
    rc = sc.lib().spchol_analyze(n, *(None if a is None else a.ctypes.data_as(C.c_void_p) for a in keep),
                                 C.byref(opts) if opts is not None else None, C.byref(h))
    if h.value:
        sc.lib().spchol_sym_destroy(h)
    return rc


def test_analyze_argument_errors():
    cp, ri = np.array([0, 2, 3]), np.array([0, 1, 1])
    assert _status(2, cp, ri) == 0
    assert _status(-1, cp, ri) == -1                           # n < 0
    assert _status(2, None, ri) == -1                          # null colptr
    assert _status(2, cp, ri, np.array([0, 0])) == -1          # not a permutation
    assert _status(2, cp, ri, np.array([0, 2])) == -1          # out of range
    assert _status(2, np.array([0, 2, 3]), np.array([1, 0, 1])) == -2   # unsorted / no diagonal
    assert _status(2, np.array([0, 1, 2]), np.array([0, 0])) == -2      # upper entry
    assert _status(2, np.array([0, 2, 2]), np.array([0, 1])) == -2      # missing diagonal col 1
    assert _status(2, np.array([0, 3, 4]), np.array([0, 1, 1, 1])) == -2  # duplicate
    from paper_2409_14009_amd import _capi
    bad = _capi.Options(0, 0, 40, 0, 0)
    assert _status(2, cp, ri, None, bad) == -1                 # panel width not a multiple of 16
    assert "panel" in sc.lib().spchol_last_error().decode()


def test_analyze_empty_and_one():
    S = sc.SparseCholesky(0, np.array([0]), np.zeros(0, np.int64))
    assert S.info()["nsuper"] == 0
    S = sc.SparseCholesky(1, np.array([0, 1]), np.array([0]))
    inf = S.info()
    assert inf["nsuper"] == 1 and inf["flops_alg"] == 1.0


def _compare_structure(n, cp, ri, perm, mode, z):
    S = sc.SparseCholesky(n, cp, ri, perm, mode, z)
    e = S.export()
    o = oracle.Symbolic(n, cp, ri, perm, mode, z)
    assert np.array_equal(e["parent"], o.parent)
    assert np.array_equal(e["count"], o.count)
    assert np.array_equal(e["super_ptr"], o.sptr)
    assert np.array_equal(e["sparent"], o.sparent)
    assert np.array_equal(e["row_ptr"], o.srptr)
    assert np.array_equal(e["row_idx"], o.srow)
    assert np.array_equal(e["pair_J"], o.pair_J)
    assert np.array_equal(e["pair_P"], o.pair_P)
    assert np.array_equal(e["pair_a0"], o.pair_a0)
    assert np.array_equal(e["relind_ptr"], o.relptr)
    assert np.array_equal(e["relind"], o.rel)
    inf = S.info()
    assert inf["flops_alg"] == o.flops()
    assert inf["nnz_l"] == o.nnzL
    # levels: leaves 0, parent above all children
    lev = e["level"]
    for J in range(inf["nsuper"]):
        P = e["sparent"][J]
        if P >= 0:
            assert lev[P] > lev[J]
    return S


def test_fig1_structure_bit_exact(fig1_pattern):
    n, cp, ri = fig1_pattern
    for mode in (0, 1):
        _compare_structure(n, cp, ri, None, mode, 0)
    S = sc.SparseCholesky(n, cp, ri, None, 1, 0)
    e = S.export()
    # relind(J1, J3) = [4, 3, 1], relind(J3, J6) = [2, 1, 0], relind(J1, J6) = [1]
    def rel(J, P):
        t = np.nonzero((e["pair_J"] == J) & (e["pair_P"] == P))[0][0]
        return e["relind"][e["relind_ptr"][t]:e["relind_ptr"][t + 1]].tolist()
    assert rel(0, 2) == [4, 3, 1] and rel(2, 5) == [2, 1, 0] and rel(0, 5) == [1]


@pytest.mark.parametrize("seed", range(16))
def test_random_structure_bit_exact(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    n, cp, ri, vv = gen.random_spd(n, rng.uniform(0.01, 0.15), rng)
    perm = rng.permutation(n)
    _compare_structure(n, cp, ri, perm, int(rng.integers(0, 2)), int(rng.integers(0, 9)))


@pytest.mark.parametrize("cfg,side", [(0, 32), (1, 12), (2, 6), (4, 14)])
@pytest.mark.parametrize("mode,z", [(0, 0), (1, 0), (0, 8)])
def test_config_structure_bit_exact(cfg, side, mode, z):
    p = gen.make_config(cfg, side=side)
    _compare_structure(p.n, p.colptr, p.rowind, p.perm, mode, z)


def test_full_size_config1_structure_bit_exact():
    """64^3, z = 8: the structure the benchmark factors."""
    p = gen.make_config(1)
    S = _compare_structure(p.n, p.colptr, p.rowind, p.perm, 0, 8)
    inf = S.info()
    assert inf["nsuper"] == 50996 and inf["nlevels"] == 38


def test_storage_offsets():
    p = gen.make_config(0)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 0)
    e = S.export()
    off = S.storage_offsets()
    k = np.diff(e["super_ptr"])
    m = np.diff(e["row_ptr"])
    assert np.array_equal(np.diff(off), k * m)
    assert off[-1] == S.info()["storage"]


def test_workspace_limit_fails_before_any_device_work():
    """A workspace limit below what the factor needs gives SPCHOL_ERR_OOM
    before the library allocates or enqueues anything (so the host path
    reports it even where no GPU is present); a negative limit is an
    argument error."""
    p = gen.make_config(0, side=12)
    S = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, workspace_limit=4096)
    h = C.c_void_p()
    info = C.c_int64(0)
    fake = C.c_void_p(256)  # never dereferenced: the limit check comes first
    rc = sc.lib().spchol_factor(S._h, fake, None, C.byref(h), C.byref(info))
    assert rc == -4 and not h.value
    msg = sc.lib().spchol_last_error().decode()
    assert "workspace limit of 4096 bytes" in msg
    need = int(msg.split("needs ")[1])
    st = S.info()["storage"]
    assert need > 8 * st
    from paper_2409_14009_amd import _capi
    assert _status(2, np.array([0, 2, 3]), np.array([0, 1, 1]), None, _capi.Options(0, 0, 64, 0, -1)) == -1


def test_deterministic_option_keeps_the_structure(monkeypatch):
    """The deterministic schedule changes launches, not the analysis: the
    exported structure is identical, with the option or the environment
    override."""
    p = gen.make_config(1, side=10)
    a = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8).export()
    b = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8, deterministic=True).export()
    monkeypatch.setenv("SPCHOL_DETERMINISTIC", "1")
    c = sc.SparseCholesky(p.n, p.colptr, p.rowind, p.perm, 0, 8).export()
    for k in a:
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
