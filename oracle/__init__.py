"""CPU oracle for supernodal sparse Cholesky -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  The GPU library shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, fp64, single thread, no
BLAS); this module loads it with ctypes and adds the closed-form gradients
and the backward-error norms on top of the C solve.

Pins (see ``tests/test_oracle_pins.py``): the worked example of Fig. 1, brute
force boolean elimination, closed-form special patterns, LAPACK's dense
Cholesky, L0 L0^T reconstruction, the closed-form grid-Laplacian
log-determinant, scipy's sparse LU solve and torch's dense autograd.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, no BLAS)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.oracle_symbolic.restype = C.c_void_p
        L.oracle_symbolic.argtypes = [C.c_int64, _i64p, _i64p, C.c_void_p, C.c_int32, C.c_int64,
                                      C.c_int32, C.c_int64, C.POINTER(C.c_int64)]
        L.oracle_free.argtypes = [C.c_void_p]
        L.oracle_sym_sizes.argtypes = [C.c_void_p, _i64p]
        L.oracle_sym_get.argtypes = [C.c_void_p] + [C.c_void_p] * 14
        L.oracle_factor.restype = C.c_int64
        L.oracle_factor.argtypes = [C.c_void_p, _f64p, C.c_int32, C.c_int64, _f64p]
        L.oracle_solve.argtypes = [C.c_void_p, _f64p, C.c_void_p, C.c_int64, C.c_int64]
        L.oracle_logdet.restype = C.c_double
        L.oracle_logdet.argtypes = [C.c_void_p, _f64p]
        L.oracle_flops.restype = C.c_double
        L.oracle_flops.argtypes = [C.c_void_p, C.c_int64]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


class Symbolic:
    """Structure of L for C = P A P^T (oracle side).

    Attributes (numpy int64 unless noted): pinv, parent, count, lptr, lrow
    (column structures, diagonal first), sptr (nsuper+1), sparent, srptr,
    srow (row lists), pair_J, pair_P, pair_a0, relptr, rel (int32; the
    paper's from-the-bottom convention).
    """

    def __init__(self, n, colptr, rowind, perm=None, snode_mode=0, amalg_z=0, amalg_rule=0, amalg_cap_percent=25):
        L = lib()
        colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        rowind = np.ascontiguousarray(rowind, dtype=np.int64)
        self._perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
        st = C.c_int64(0)
        h = L.oracle_symbolic(int(n), colptr, rowind if rowind.size else np.zeros(1, np.int64),
                              _ptr(self._perm), int(snode_mode), int(amalg_z), int(amalg_rule),
                              int(amalg_cap_percent), C.byref(st))
        if not h:
            raise OracleError(f"oracle_symbolic failed with status {st.value}")
        self._h = h
        self.n = int(n)
        self.nnzA = int(colptr[-1]) if len(colptr) else 0
        sz = np.zeros(6, np.int64)
        L.oracle_sym_sizes(h, sz)
        n_, nnzL, ns, nsr, npairs, nrel = (int(x) for x in sz)
        self.nnzL, self.nsuper, self.npairs = nnzL, ns, npairs
        mk = lambda k: np.zeros(max(k, 0), np.int64)
        self.pinv, self.parent, self.count = mk(n_), mk(n_), mk(n_)
        self.lptr, self.lrow = mk(n_ + 1), mk(nnzL)
        self.sptr, self.sparent, self.srptr, self.srow = mk(ns + 1), mk(ns), mk(ns + 1), mk(nsr)
        self.pair_J, self.pair_P, self.pair_a0, self.relptr = mk(npairs), mk(npairs), mk(npairs), mk(npairs + 1)
        self.rel = np.zeros(nrel, np.int32)
        L.oracle_sym_get(h, *[_ptr(a) for a in (self.pinv, self.parent, self.count, self.lptr, self.lrow,
                                                  self.sptr, self.sparent, self.srptr, self.srow,
                                                  self.pair_J, self.pair_P, self.pair_a0, self.relptr,
                                                  self.rel)])
        self.perm = np.argsort(self.pinv) if n_ else np.zeros(0, np.int64)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_free(h)
            self._h = None

    # --- convenience views -------------------------------------------------
    def supernode_rows(self, J):
        return self.srow[self.srptr[J]:self.srptr[J + 1]]

    def supernode_cols(self, J):
        return np.arange(self.sptr[J], self.sptr[J + 1])

    def relind(self, J, P):
        """relind(J, P) as an int array (from-the-bottom convention)."""
        idx = np.nonzero((self.pair_J == J) & (self.pair_P == P))[0]
        if idx.size == 0:
            return None
        t = int(idx[0])
        return self.rel[self.relptr[t]:self.relptr[t + 1]]

    def flops(self, ncols: int = -1) -> float:
        """sum_j c_j^2 over the first ncols columns (all by default)."""
        return float(lib().oracle_flops(self._h, int(ncols)))

    # --- numeric -----------------------------------------------------------
    def factor(self, vals, variant: int = 0, ncols: int = -1) -> "Factor":
        """variant 0 left-looking, 1 up-looking.  ncols >= 0 (left-looking)
        computes only the first ncols columns, which are then final."""
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        if vals.size != self.nnzA:
            raise OracleError("values length does not match the pattern")
        lv = np.zeros(max(self.nnzL, 1), np.float64)
        info = int(lib().oracle_factor(self._h, vals if vals.size else np.zeros(1), int(variant), int(ncols), lv))
        f = Factor(self, lv[: self.nnzL], info, vals)
        f.ncols = self.n if ncols < 0 else min(int(ncols), self.n)
        return f


class Factor:
    def __init__(self, sym: Symbolic, lv, info, vals):
        self.sym, self.lv, self.info, self.vals = sym, lv, info, vals

    def require_ok(self):
        if getattr(self, "ncols", self.sym.n) < self.sym.n:
            raise OracleError("partial factor: only the leading columns were computed")
        if self.info != 0:
            raise OracleError(f"not positive definite at (permuted, 1-based) column {self.info}")

    def L_csc(self) -> sp.csc_matrix:
        s = self.sym
        return sp.csc_matrix((self.lv, s.lrow, s.lptr), shape=(s.n, s.n))

    def solve(self, B) -> np.ndarray:
        self.require_ok()
        B = np.array(B, dtype=np.float64, copy=True)
        one = B.ndim == 1
        X = np.asfortranarray(B.reshape(self.sym.n, -1))
        Xc = np.ascontiguousarray(X.T)  # rows = rhs, each contiguous (ld = n)
        lib().oracle_solve(self.sym._h, self.lv if self.lv.size else np.zeros(1),
                           _ptr(Xc), Xc.shape[0], self.sym.n)
        X = Xc.T
        return X.ravel() if one else np.asfortranarray(X)

    def logdet(self) -> float:
        self.require_ok()
        return float(lib().oracle_logdet(self.sym._h, self.lv if self.lv.size else np.zeros(1)))

    def diag(self) -> np.ndarray:
        return self.lv[self.sym.lptr[:-1]]


# --------------------------------------------------------------------------
# Closed-form reverse mode and error norms on top of the oracle solve.
# --------------------------------------------------------------------------

def full_matrix(n, colptr, rowind, vals) -> sp.csr_matrix:
    """Symmetric A from its stored lower triangle."""
    Lw = sp.csc_matrix((vals, rowind, colptr), shape=(n, n))
    return (Lw + Lw.T - sp.diags(Lw.diagonal())).tocsr()


def entry_coords(colptr, rowind):
    """(row, col) of every stored lower entry, in storage order."""
    n = len(colptr) - 1
    cols = np.repeat(np.arange(n), np.diff(colptr))
    return np.asarray(rowind, np.int64), cols


def grad_logdet(fac: Factor, colptr, rowind, entries=None) -> np.ndarray:
    """d logdet(A) / d a_ij for stored lower entries (tied symmetric
    parameter): 2 (A^-1)_ij off the diagonal, (A^-1)_ii on it.  (A^-1)_ij
    comes from a solve with the unit vector e_j.  `entries` selects stored
    positions (default: all, only sensible for small n)."""
    r, c = entry_coords(colptr, rowind)
    if entries is None:
        entries = np.arange(len(r))
    n = fac.sym.n
    out = np.zeros(len(entries))
    cache = {}
    for t, p in enumerate(entries):
        i, j = int(r[p]), int(c[p])
        if j not in cache:
            e = np.zeros(n)
            e[j] = 1.0
            cache[j] = fac.solve(e)
        z = cache[j][i]
        out[t] = z if i == j else 2.0 * z
    return out


def grad_solve(fac: Factor, colptr, rowind, x, xbar, entries=None):
    """Reverse mode of x = A^-1 b for cotangent xbar (n x nrhs):
    lam = A^-1 xbar, Abar_ij = -(lam_i x_j + lam_j x_i) (i != j),
    -lam_i x_i (i == j), summed over RHS columns; bbar = lam."""
    x = np.asarray(x, np.float64).reshape(fac.sym.n, -1)
    xbar = np.asarray(xbar, np.float64).reshape(fac.sym.n, -1)
    lam = fac.solve(xbar).reshape(fac.sym.n, -1)
    r, c = entry_coords(colptr, rowind)
    if entries is not None:
        r, c = r[entries], c[entries]
    g = -(lam[r] * x[c]).sum(axis=1)
    off = r != c
    g[off] -= (lam[c[off]] * x[r[off]]).sum(axis=1)
    return g, lam


def backward_error(A: sp.csr_matrix, X, B):
    """Normwise backward error per RHS column,
    eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), and the
    componentwise max_i |r_i| / (|A||x| + |b|)_i."""
    X = np.asarray(X, np.float64).reshape(A.shape[0], -1)
    B = np.asarray(B, np.float64).reshape(A.shape[0], -1)
    R = B - A @ X
    Anorm = abs(A).sum(axis=1).max() if A.shape[0] else 0.0
    eta = np.abs(R).max(axis=0) / (Anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0))
    den = abs(A) @ np.abs(X) + np.abs(B)
    with np.errstate(divide="ignore", invalid="ignore"):
        comp = np.where(den > 0, np.abs(R) / den, 0.0).max(axis=0)
    return eta, comp


def timed_factor(sym: Symbolic, vals, repeats: int = 1):
    """(seconds, Factor) -- median of `repeats` oracle factorizations."""
    ts, fac = [], None
    for _ in range(repeats):
        t0 = time.perf_counter()
        fac = sym.factor(vals)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), fac
