"""Helpers for the GPU parity tests (host-side conversions and norms)."""
import numpy as np
import scipy.sparse as sp


def storage_to_csc(export, off, Lst, n):
    """Supernodal storage (host numpy, layout of spchol_sym_storage) -> CSC of
    the lower factor with every stored lower-trapezoid entry (explicit zeros
    of amalgamation included), plus the max |entry| found in the upper
    triangles of the diagonal blocks (must be 0)."""
    spr, rp, ri = export["super_ptr"], export["row_ptr"], export["row_idx"]
    rows, cols, vals = [], [], []
    upper_max = 0.0
    for J in range(len(spr) - 1):
        f, k = int(spr[J]), int(spr[J + 1] - spr[J])
        R = ri[rp[J]:rp[J + 1]]
        m = len(R)
        blk = Lst[off[J]:off[J] + k * m].reshape(k, m)  # blk[c] = column c
        cc, pp = np.nonzero(np.arange(m)[None, :] >= np.arange(k)[:, None])
        rows.append(R[pp])
        cols.append(f + cc)
        vals.append(blk[cc, pp])
        cu, pu = np.nonzero(np.arange(m)[None, :] < np.arange(k)[:, None])
        if cu.size:
            upper_max = max(upper_max, float(np.abs(blk[cu, pu]).max()))
    if rows:
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    else:
        rows = cols = np.zeros(0, np.int64)
        vals = np.zeros(0)
    L = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    return L, upper_max


def compare_factor(Lg, Lo, Cdiag):
    """Split the GPU factor Lg into the oracle's structure and the rest.
    Returns (max |Lg - Lo| / sqrt(C_ii) on the oracle structure,
    max |Lg| off the oracle structure, relative Frobenius difference)."""
    Lo = Lo.tocsc()
    pat = Lo.copy()
    pat.data = np.ones_like(pat.data)
    on = Lg.multiply(pat)
    off = Lg - on
    D = (on - Lo).tocoo()
    scale = np.sqrt(np.abs(Cdiag))
    elt = float((np.abs(D.data) / scale[D.row]).max()) if D.nnz else 0.0
    offmax = float(np.abs(off.data).max()) if off.nnz else 0.0
    fro = float(sp.linalg.norm(on - Lo) / max(sp.linalg.norm(Lo), 1e-300))
    return elt, offmax, fro


def permuted_matrix(A_full, perm):
    return A_full[perm][:, perm].tocsc()


def residual_rel(Cm, L):
    """||C - L L^T||_F / ||C||_F, exact on the pattern (small n)."""
    R = Cm - L @ L.T
    return float(sp.linalg.norm(R) / sp.linalg.norm(Cm))
