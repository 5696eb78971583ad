"""MI355X-native supernodal sparse Cholesky (right-looking, Sec. II-A).

Thin Python binding over the C ABI of ``libspchol.so`` (include/spchol.h):
argument marshalling only.  Every numeric step runs in the library's HIP
kernels; torch supplies device memory and streams.  If the library is not
built, using it raises ``LibraryMissing`` -- there is no CPU fallback.

    S = SparseCholesky(n, colptr, rowind, perm, amalg_max_zeros=8)
    F = S.factor(vals_dev)           # torch.float64 CUDA tensor, nnz(A) values
    x = F.solve(b_dev)               # (n,) or (n, nrhs)
    ld = F.logdet()
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi as capi
from ._capi import LibraryMissing

__all__ = ["SparseCholesky", "BatchCholesky", "Factor", "Graph", "SpcholError", "NotPositiveDefinite",
           "LibraryMissing", "version", "lib", "logdet_solve"]


def lib():
    return capi.lib()


def version() -> str:
    return capi.lib().spchol_version().decode()


class SpcholError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{capi.STATUS.get(status, status)}: {message}")
        self.status = status


class NotPositiveDefinite(SpcholError):
    def __init__(self, status, message, info):
        super().__init__(status, message)
        self.info = info


def _check(rc):
    if rc != 0:
        msg = capi.lib().spchol_last_error()
        raise SpcholError(rc, msg.decode() if msg else "")


def _hptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev_f64(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{what} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return C.c_void_p(t.data_ptr())


PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2}


def _precision(p):
    if isinstance(p, int):
        return p
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"unknown update precision {p!r}") from None


def _update_method(u):
    """"rl" / "rlb" (or 0 / 1): how a supernode's update reaches its ancestors."""
    m = {"rl": 0, "rlb": 1, 0: 0, 1: 1}
    if u not in m:
        raise ValueError(f"unknown update method {u!r}")
    return m[u]


def order_nd(n, colptr, rowind, leaf_size=64, seed=1):
    """Nested-dissection ordering of a sparse symmetric pattern (host; the
    library's multilevel bisection, spchol_order_nd): perm[k] = the original
    index eliminated k-th."""
    cp = np.ascontiguousarray(colptr, dtype=np.int64)
    ri = np.ascontiguousarray(rowind, dtype=np.int64)
    perm = np.zeros(int(n), np.int64)
    _check(capi.lib().spchol_order_nd(int(n), _hptr(cp), _hptr(ri), int(leaf_size), int(seed), _hptr(perm)))
    return perm


class SparseCholesky:
    """Symbolic analysis of a sparse SPD pattern (host), bound to the device
    of its first factorization."""

    def __init__(self, n, colptr, rowind, perm=None, snode_mode=0, amalg_max_zeros=0, panel_width=64,
                 deterministic=False, workspace_limit=0, amalg_rule=0, amalg_cap_percent=25, update_method=0,
                 partition_refinement=False):
        L = capi.lib()
        self.n = int(n)
        self._colptr = np.ascontiguousarray(colptr, dtype=np.int64)
        self._rowind = np.ascontiguousarray(rowind, dtype=np.int64)
        self._perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
        opts = capi.Options(int(snode_mode), int(amalg_max_zeros), int(panel_width), int(bool(deterministic)),
                            int(workspace_limit), int(amalg_rule), int(amalg_cap_percent),
                            _update_method(update_method), int(bool(partition_refinement)))
        h = C.c_void_p()
        _check(L.spchol_analyze(self.n, _hptr(self._colptr), _hptr(self._rowind), _hptr(self._perm),
                                C.byref(opts), C.byref(h)))
        self._h = h
        self.nnz_a = int(self._colptr[-1]) if self._colptr.size else 0

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().spchol_sym_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        s = capi.SymInfo()
        _check(capi.lib().spchol_sym_info(self._h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_}

    def export(self) -> dict:
        """Structure arrays (host numpy), names as in spchol_sym_export."""
        inf = self.info()
        n, ns, npairs = inf["n"], inf["nsuper"], inf["npairs"]
        out = dict(parent=np.zeros(n, np.int64), count=np.zeros(n, np.int64),
                   super_ptr=np.zeros(ns + 1, np.int64), sparent=np.zeros(ns, np.int64),
                   row_ptr=np.zeros(ns + 1, np.int64), row_idx=np.zeros(inf["nrows_total"], np.int64),
                   pair_J=np.zeros(npairs, np.int64), pair_P=np.zeros(npairs, np.int64),
                   pair_a0=np.zeros(npairs, np.int64), relind_ptr=np.zeros(npairs + 1, np.int64),
                   relind=np.zeros(inf["nrelind"], np.int32), level=np.zeros(ns, np.int64))
        keys = ["parent", "count", "super_ptr", "sparent", "row_ptr", "row_idx", "pair_J", "pair_P",
                "pair_a0", "relind_ptr", "relind", "level"]
        _check(capi.lib().spchol_sym_export(self._h, *[_hptr(out[k]) for k in keys]))
        return out

    def batch_info(self):
        """(count, col_off[count+1], nz_off[count+1]) of a batch handle."""
        cnt = C.c_int32(0)
        _check(capi.lib().spchol_batch_info(self._h, C.byref(cnt), None, None))
        co = np.zeros(cnt.value + 1, np.int64)
        no = np.zeros(cnt.value + 1, np.int64)
        _check(capi.lib().spchol_batch_info(self._h, C.byref(cnt), _hptr(co), _hptr(no)))
        return cnt.value, co, no

    def perm(self) -> np.ndarray:
        """The elimination order the analysis used (the given perm, or the
        partition-refined one)."""
        out = np.zeros(self.n, np.int64)
        _check(capi.lib().spchol_sym_perm(self._h, _hptr(out)))
        return out

    def storage_offsets(self) -> np.ndarray:
        inf = self.info()
        off = np.zeros(inf["nsuper"] + 1, np.int64)
        _check(capi.lib().spchol_sym_storage(self._h, _hptr(off)))
        return off

    def factor_streamed(self, vals, device_budget=256 << 20, host_threshold=600000, host_threads=0, stream=None,
                        check=True):
        """Host-resident factorization (spchol_factor_streamed): vals is a
        host float64 array; returns (L storage as a host numpy array, info,
        stats dict).  Supernodes with k * m below host_threshold are done
        on the host, the others on the device within device_budget bytes."""
        v = np.ascontiguousarray(vals, dtype=np.float64)
        if v.size != self.nnz_a:
            raise ValueError("vals has the wrong length")
        L = np.empty(max(int(self.info()["storage"]), 1), np.float64)
        opts = capi.StreamOptions(int(device_budget), int(host_threshold), int(host_threads), 0)
        st = capi.StreamStats()
        info = C.c_int64(0)
        if stream is None:
            import torch
            sp = _stream_ptr(None) if torch.cuda.is_available() else C.c_void_p(None)
        else:
            sp = _stream_ptr(stream)
        rc = capi.lib().spchol_factor_streamed(self._h, _hptr(v) if v.size else None, C.byref(opts), sp, _hptr(L),
                                               C.byref(info), C.byref(st))
        stats = {name: getattr(st, name) for name, _ in st._fields_ if name != "reserved"}
        if rc == -3 and check:
            raise NotPositiveDefinite(rc, capi.lib().spchol_last_error().decode(), int(info.value))
        if rc != -3:
            _check(rc)
        return L[: int(self.info()["storage"])], int(info.value), stats

    def factor(self, vals, stream=None, check=True, precision="f64") -> "Factor":
        """Numeric factorization of the values `vals` (float64 CUDA tensor in
        the pattern's entry order).  precision: "f64", "f32" or "bf16" for the
        update products (the diagonal-block Cholesky and the solves stay fp64).
        Raises NotPositiveDefinite (with .info, the 1-based permuted column)
        when check is set."""
        if vals.numel() != self.nnz_a:
            raise ValueError("vals has the wrong length")
        h = C.c_void_p()
        info = C.c_int64(0)
        rc = capi.lib().spchol_factor_prec(self._h, _dev_f64(vals, "vals"), _precision(precision),
                                           _stream_ptr(stream), C.byref(h), C.byref(info))
        F = Factor(self, h) if h.value else None
        if rc == -3:
            if F is not None:
                F.info = int(info.value)
            if check:
                raise NotPositiveDefinite(rc, capi.lib().spchol_last_error().decode(), int(info.value))
            return F
        _check(rc)
        F.info = 0
        return F


class BatchCholesky(SparseCholesky):
    """Symbolic analysis of many independent matrices as one block-diagonal
    matrix: `mats` is a list of (n, colptr, rowind, perm) tuples.  Values
    and right-hand sides are the concatenation of the per-matrix ones."""

    def __init__(self, mats, snode_mode=0, amalg_max_zeros=0, panel_width=64, deterministic=False,
                 workspace_limit=0, amalg_rule=0, amalg_cap_percent=25, update_method=0, partition_refinement=False):
        L = capi.lib()
        self._keep = []
        cnt = len(mats)
        ns = np.array([int(m[0]) for m in mats], np.int64)
        cps = [np.ascontiguousarray(m[1], np.int64) for m in mats]
        ris = [np.ascontiguousarray(m[2], np.int64) for m in mats]
        pms = [None if m[3] is None else np.ascontiguousarray(m[3], np.int64) for m in mats]
        self._keep = [ns, cps, ris, pms]
        arr = lambda xs: (C.c_void_p * max(cnt, 1))(*[None if x is None else x.ctypes.data for x in xs])
        self._pa = (arr(cps), arr(ris), arr(pms))
        opts = capi.Options(int(snode_mode), int(amalg_max_zeros), int(panel_width), int(bool(deterministic)),
                            int(workspace_limit), int(amalg_rule), int(amalg_cap_percent),
                            _update_method(update_method), int(bool(partition_refinement)))
        h = C.c_void_p()
        _check(L.spchol_batch_analyze(cnt, _hptr(ns), C.cast(self._pa[0], C.c_void_p), C.cast(self._pa[1], C.c_void_p),
                                      C.cast(self._pa[2], C.c_void_p), C.byref(opts), C.byref(h)))
        self._h = h
        self.n = int(ns.sum())
        self.nnz_a = int(sum(int(c[-1]) for c in cps))
        self.count = cnt


class Graph:
    """A captured factorization (+ solve) replayed as one launch."""

    def __init__(self, factor, h):
        self.factor = factor
        self._h = h

    def replay(self, stream=None):
        _check(capi.lib().spchol_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().spchol_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """Numeric factor held in device memory."""

    def __init__(self, sym: SparseCholesky, h):
        self.sym = sym
        self._h = h
        self.info = 0
        self.last_refine_path = 0

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().spchol_num_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refactor(self, vals, stream=None, check=True, precision=None) -> int:
        info = C.c_int64(0)
        if precision is None:
            rc = capi.lib().spchol_refactor(self._h, _dev_f64(vals, "vals"), _stream_ptr(stream), C.byref(info))
        else:
            rc = capi.lib().spchol_refactor_prec(self._h, _dev_f64(vals, "vals"), _precision(precision),
                                                 _stream_ptr(stream), C.byref(info))
        self.info = int(info.value)
        if rc == -3 and not check:
            return self.info
        if rc == -3:
            raise NotPositiveDefinite(rc, capi.lib().spchol_last_error().decode(), self.info)
        _check(rc)
        return 0

    def solve_(self, Bt, stream=None):
        """In place on a (nrhs, n) contiguous float64 CUDA tensor, i.e. an
        n x nrhs column-major block with leading dimension n."""
        nrhs = Bt.shape[0] if Bt.dim() == 2 else 1
        _check(capi.lib().spchol_solve(self._h, _dev_f64(Bt, "B"), nrhs, self.sym.n, _stream_ptr(stream)))
        return Bt

    def solve_noalloc_(self, Bt, stream=None):
        """solve_ with the library's static per-GPU work array instead of the
        handle's buffers (spchol_solve_noalloc: allocates nothing; n * nrhs
        at most 2^21; calls overlapping on one GPU race)."""
        nrhs = Bt.shape[0] if Bt.dim() == 2 else 1
        _check(capi.lib().spchol_solve_noalloc(self._h, _dev_f64(Bt, "B"), nrhs, self.sym.n, _stream_ptr(stream)))
        return Bt

    def solve(self, B, stream=None):
        """Return A^{-1} B for B of shape (n,) or (n, nrhs)."""
        if B.dim() == 1:
            X = B.contiguous().clone()
            return self.solve_(X.view(1, -1), stream).view(-1)
        Xt = B.t().contiguous()
        self.solve_(Xt, stream)
        return Xt.t()

    def refine_(self, vals, Bt, Xt, tol=1e-12, max_iter=10, stream=None, check=True):
        """Iterative refinement on (nrhs, n) contiguous tensors (column-major
        n x nrhs blocks): Xt <- A^{-1} Bt.  Returns (berr per RHS, iterations);
        `last_refine_path` is then 0 (refinement alone) or 1 (it stalled and
        the remaining corrections were preconditioned conjugate-gradient
        steps).  Raises SpcholError(SPCHOL_ERR_NOCONV) when check is set and
        the tolerance is not reached."""
        nrhs = Bt.shape[0] if Bt.dim() == 2 else 1
        berr = (C.c_double * max(nrhs, 1))()
        iters = C.c_int32(0)
        path = C.c_int32(0)
        rc = capi.lib().spchol_refine(self._h, _dev_f64(vals, "vals"), _dev_f64(Bt, "B"), _dev_f64(Xt, "X"),
                                      nrhs, self.sym.n, self.sym.n, float(tol), int(max_iter), _stream_ptr(stream),
                                      berr, C.byref(iters), C.byref(path))
        self.last_refine_path = int(path.value)
        out = ([berr[c] for c in range(nrhs)], int(iters.value))
        if rc == -6 and not check:
            return out
        _check(rc)
        return out

    def berr_(self, vals, Bt, Xt, stream=None):
        """Normwise backward error per right-hand side of the (nrhs, n)
        contiguous solution block Xt for the block Bt (fp64, original A)."""
        nrhs = Bt.shape[0] if Bt.dim() == 2 else 1
        out = (C.c_double * max(nrhs, 1))()
        _check(capi.lib().spchol_berr(self._h, _dev_f64(vals, "vals"), _dev_f64(Bt, "B"), _dev_f64(Xt, "X"), nrhs,
                                      self.sym.n, self.sym.n, _stream_ptr(stream), out))
        return [out[c] for c in range(nrhs)]

    def refine(self, vals, B, tol=1e-12, max_iter=10, stream=None, check=True):
        """X = A^{-1} B by iterative refinement with this factor; B of shape
        (n,) or (n, nrhs).  Returns (X, berr list, iterations)."""
        import torch
        one = B.dim() == 1
        Bt = (B.view(1, -1) if one else B.t()).contiguous()
        Xt = torch.empty_like(Bt)
        berr, it = self.refine_(vals, Bt, Xt, tol, max_iter, stream, check)
        X = Xt.view(-1) if one else Xt.t()
        return X, berr, it

    def backward(self, X, Xbar, gbar_logdet, stream=None):
        """Reverse mode of (logdet, X = A^{-1} B): returns (Abar, Bbar) for
        the stored lower values of A and for B.  X, Xbar: (n,) or (n, nrhs)
        float64 CUDA tensors (Xbar may be None); gbar_logdet: float."""
        import torch
        n = self.sym.n
        Abar = torch.empty(max(self.sym.nnz_a, 1), dtype=torch.float64, device="cuda")[: self.sym.nnz_a]
        if Xbar is None or X is None:
            _check(capi.lib().spchol_backward(self._h, None, None, 0, max(n, 1), float(gbar_logdet),
                                              C.c_void_p(Abar.data_ptr()), None, _stream_ptr(stream)))
            return Abar, None
        one = X.dim() == 1
        Xt = (X.view(1, -1) if one else X.t()).contiguous()
        Gt = (Xbar.view(1, -1) if one else Xbar.t()).contiguous()
        Bt = torch.empty_like(Xt)
        nrhs = Xt.shape[0]
        _check(capi.lib().spchol_backward(self._h, _dev_f64(Xt, "X"), _dev_f64(Gt, "Xbar"), nrhs, n,
                                          float(gbar_logdet), C.c_void_p(Abar.data_ptr()),
                                          _dev_f64(Bt, "Bbar"), _stream_ptr(stream)))
        Bbar = Bt.view(-1) if one else Bt.t()
        return Abar, Bbar

    def logdet_batch(self, stream=None):
        """Per-matrix log-determinants of a batch (float64 CUDA tensor)."""
        import torch
        cnt = self.sym.batch_info()[0]
        out = torch.empty(cnt, dtype=torch.float64, device="cuda")
        _check(capi.lib().spchol_logdet_batch(self._h, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def status(self, stream=None) -> int:
        """Pivot status of the last factorization enqueued (0 = SPD)."""
        info = C.c_int64(0)
        rc = capi.lib().spchol_info(self._h, C.byref(info), _stream_ptr(stream))
        if rc not in (0, -3):
            _check(rc)
        return int(info.value)

    def capture(self, vals, Bt=None, stream=None) -> Graph:
        """Capture factorization (vals None: none) + in-place solve of the
        (nrhs, n) tensor Bt (None: none) as a hipGraph on `stream` (default:
        torch's current stream, which must not be the null stream)."""
        h = C.c_void_p()
        nrhs = 0 if Bt is None else (Bt.shape[0] if Bt.dim() == 2 else 1)
        bp = None if Bt is None else _dev_f64(Bt, "B")
        vp = None if vals is None else _dev_f64(vals, "vals")
        _check(capi.lib().spchol_graph_create(self._h, vp, bp, nrhs, max(self.sym.n, 1),
                                              _stream_ptr(stream), C.byref(h)))
        return Graph(self, h)

    def selinv(self, stream=None):
        """Selected inverse of C = P A P^T on the supernodal pattern, in the
        storage layout of L (float64 CUDA tensor)."""
        import torch
        n = int(self.sym.info()["storage"])
        out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        _check(capi.lib().spchol_selinv_export(self._h, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out[:n]

    def logdet(self, stream=None) -> float:
        out = C.c_double(0.0)
        _check(capi.lib().spchol_logdet(self._h, C.byref(out), _stream_ptr(stream)))
        return float(out.value)

    def profile(self, enable: bool = True, alone: bool = False):
        """Start (clearing earlier records) or stop per-launch event timing;
        alone: every launch runs by itself on the caller's stream (no second
        stream), so each record is that launch's own duration."""
        _check(capi.lib().spchol_profile(self._h, (2 if alone else 1) if enable else 0))

    def profile_read(self) -> dict:
        """Per kernel kind: launches, ms, flops, bytes summed over the records
        since profile(True); synchronizes and clears them."""
        arr = (capi.KernelStat * len(capi.KERNEL_KINDS))()
        _check(capi.lib().spchol_profile_read(self._h, arr))
        return {name: dict(launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops, bytes=arr[i].bytes)
                for i, name in enumerate(capi.KERNEL_KINDS)}

    def profile_launches(self) -> list:
        """The records since profile(True) one by one, in launch order: kind
        name, schedule level (-1 outside the level schedule), side (1: second
        stream), ms, flops, bytes; synchronizes and clears them."""
        cnt = C.c_int64(0)
        _check(capi.lib().spchol_profile_launches(self._h, None, 0, C.byref(cnt)))
        arr = (capi.LaunchRecord * max(cnt.value, 1))()
        _check(capi.lib().spchol_profile_launches(self._h, arr, cnt.value, C.byref(cnt)))
        return [dict(kind=capi.KERNEL_KINDS[r.kind], level=r.level, side=r.side, ms=r.ms, flops=r.flops,
                     bytes=r.bytes) for r in arr[:cnt.value]]

    def storage(self, stream=None):
        """Copy of the supernodal storage of L (float64 CUDA tensor)."""
        import torch
        n = int(self.sym.info()["storage"])
        out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        _check(capi.lib().spchol_num_export(self._h, C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out[:n]


def _autograd():
    import torch

    class LogdetSolve(torch.autograd.Function):
        """(logdet(A), A^{-1} b) as a differentiable function of the stored
        lower values of A and of b; the backward pass is the library's
        reverse-mode kernels (selected inversion + adjoint solve)."""

        @staticmethod
        def forward(ctx, vals, b, sym, precision):
            F = sym.factor(vals.detach(), precision=precision)
            x = F.solve(b.detach())
            ld = F.logdet()
            ctx.F = F
            ctx.save_for_backward(x)
            return torch.tensor(ld, dtype=torch.float64, device=vals.device), x

        @staticmethod
        def backward(ctx, gld, gx):
            (x,) = ctx.saved_tensors
            gl = float(gld) if gld is not None else 0.0
            Abar, Bbar = ctx.F.backward(x, gx.contiguous() if gx is not None else None, gl)
            if Bbar is None:
                Bbar = torch.zeros_like(x)
            return Abar, Bbar, None, None

    return LogdetSolve


_LogdetSolve = None


def logdet_solve(sym: SparseCholesky, vals, b, precision="f64"):
    """Differentiable (logdet(A), x = A^{-1} b) for the pattern analysed in
    `sym`; gradients flow to `vals` (stored lower entries) and `b`."""
    global _LogdetSolve
    if _LogdetSolve is None:
        _LogdetSolve = _autograd()
    return _LogdetSolve.apply(vals, b, sym, precision)
