"""Seeded synthetic inputs: SPD grid operators, geometric nested dissection, RHS.

This module builds the *inputs* that both the GPU library and the CPU oracle
consume.  It holds none of the factorization's arithmetic: it only assembles
matrices (lower-triangular CSC, original ordering), a fill-reducing ordering
(passed to the method as an input permutation) and right-hand sides.

The paper measures on SuiteSparse matrices ordered with METIS nested
dissection (Sec. IV-A).  Neither is available here, so the workloads are the
grid families below, with a deterministic geometric nested dissection standing
in for METIS.  No SuiteSparse item is reproduced.

Conventions
-----------
* Nodes of a grid of shape (nx, ny[, nz]) are numbered x fastest:
  ``u = x + nx*y + nx*ny*z``.
* Undirected edges are enumerated by node index, then by stencil offset in
  increasing linear-offset order (the "forward half" of the stencil), and
  random per-edge values are drawn in that order.
* A matrix is returned as the lower triangle (diagonal included) in CSC form:
  ``colptr`` (n+1, int64), ``rowind`` (int64, strictly increasing inside a
  column), ``vals`` (float64, same order as ``rowind``).
* ``perm[k]`` is the original index eliminated k-th.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import itertools

import numpy as np
import scipy.sparse as sp

BASE_SEED = 20240914

__all__ = [
    "Problem", "BASE_SEED", "stencil_offsets", "grid_edges", "nested_dissection",
    "laplacian_from_edges", "grid_laplacian", "elasticity_27pt", "gaussian_random_field",
    "grf_laplacian", "random_spd", "make_config", "make_batch", "expand_block_perm",
    "full_from_lower",
]


@dataclass
class Problem:
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    vals: np.ndarray
    perm: np.ndarray
    B: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------

def stencil_offsets(dim: int, kind: str) -> list[tuple[int, ...]]:
    """Forward half of a stencil, ordered by increasing linear offset.

    kind: "star" (5-point in 2D, 7-point in 3D) or "box" (9-point / 27-point).
    """
    if kind == "star":
        offs = [tuple(1 if a == d else 0 for a in range(dim)) for d in range(dim)]
    elif kind == "box":
        offs = [o for o in itertools.product((-1, 0, 1), repeat=dim) if any(o)]
        # keep the half whose linear offset (x fastest) is positive
        offs = [o for o in offs if _lin_sign(o) > 0]
    else:
        raise ValueError(kind)
    # sort by the linear offset for a generic large grid (x fastest):
    # dominant coordinate is the last one.
    return sorted(offs, key=lambda o: tuple(reversed(o)))


def _lin_sign(o):
    for c in reversed(o):
        if c != 0:
            return 1 if c > 0 else -1
    return 0


def grid_edges(shape, offsets):
    """All undirected grid edges (u, v), u < v, in the documented order."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    n = int(np.prod(shape))
    coords = np.indices(shape[::-1]).reshape(dim, -1)[::-1]  # coords[d][u], x fastest
    strides = np.cumprod((1,) + shape[:-1])
    us, vs, keys = [], [], []
    node = np.arange(n, dtype=np.int64)
    for oi, off in enumerate(offsets):
        ok = np.ones(n, dtype=bool)
        for d in range(dim):
            c = coords[d] + off[d]
            ok &= (c >= 0) & (c < shape[d])
        u = node[ok]
        v = u + int(np.dot(off, strides))
        us.append(u)
        vs.append(v)
        keys.append(u * len(offsets) + oi)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    order = np.argsort(np.concatenate(keys), kind="stable")
    u, v = u[order], v[order]
    assert np.all(v > u)
    return u, v


def nested_dissection(shape) -> np.ndarray:
    """Geometric nested dissection of a box grid (x fastest numbering).

    Box [lo, hi) per axis.  Split the longest axis (lowest axis index on ties)
    at mid = (lo + hi) // 2: the plane at mid is the separator, [lo, mid) the
    low side and [mid+1, hi) the high side.  Order: low side, high side, then
    the separator (lexicographic, x fastest).  Recurse down to single nodes.
    A plane separates the 5/7-point and the 9/27-point stencils alike.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    strides = np.cumprod((1,) + shape[:-1]).astype(np.int64)
    out = []

    def box_nodes(lo, hi):
        rng = [np.arange(lo[d], hi[d], dtype=np.int64) for d in range(dim)]
        # lexicographic with x fastest: iterate last axis slowest
        grids = np.meshgrid(*rng[::-1], indexing="ij")
        lin = np.zeros(grids[0].shape, dtype=np.int64)
        for d in range(dim):
            lin += grids[dim - 1 - d] * strides[d]
        return lin.ravel()

    def rec(lo, hi):
        ext = [hi[d] - lo[d] for d in range(dim)]
        if min(ext) <= 0:
            return
        if max(ext) == 1:
            out.append(np.array([int(np.dot(lo, strides))], dtype=np.int64))
            return
        ax = int(np.argmax(ext))  # first maximum -> lowest axis index on ties
        mid = (lo[ax] + hi[ax]) // 2
        lo_low, hi_low = list(lo), list(hi)
        hi_low[ax] = mid
        lo_high, hi_high = list(lo), list(hi)
        lo_high[ax] = mid + 1
        lo_sep, hi_sep = list(lo), list(hi)
        lo_sep[ax], hi_sep[ax] = mid, mid + 1
        rec(lo_low, hi_low)
        rec(lo_high, hi_high)
        out.append(box_nodes(lo_sep, hi_sep))

    rec([0] * dim, list(shape))
    perm = np.concatenate(out)
    assert perm.size == int(np.prod(shape))
    return perm


def expand_block_perm(node_perm: np.ndarray, dof: int) -> np.ndarray:
    """Node ordering -> dof ordering with the dofs of a node consecutive."""
    return (node_perm[:, None] * dof + np.arange(dof)[None, :]).ravel().astype(np.int64)


# --------------------------------------------------------------------------
# assembly (lower CSC, original ordering)
# --------------------------------------------------------------------------

def _lower_csc(n, rows, cols, vals):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsc()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int64), A.data.astype(np.float64))


def laplacian_from_edges(n, u, v, w, shift):
    """Weighted graph Laplacian + shift*I: a_uv = -w_uv, a_uu = sum_v w_uv + shift."""
    diag = np.full(n, float(shift))
    np.add.at(diag, u, w)
    np.add.at(diag, v, w)
    rows = np.concatenate([v, np.arange(n)])
    cols = np.concatenate([u, np.arange(n)])
    vals = np.concatenate([-w, diag])
    return _lower_csc(n, rows, cols, vals)


def full_from_lower(n, colptr, rowind, vals):
    """Symmetric scipy CSR matrix from its lower triangle (test helper)."""
    L = sp.csc_matrix((vals, rowind, colptr), shape=(n, n))
    D = sp.diags(L.diagonal())
    return (L + L.T - D).tocsr()


def grid_laplacian(shape, rng=None, weights="uniform", lo=0.5, hi=1.5, shift=1e-2,
                   kind="star"):
    """Grid graph Laplacian.  weights: "uniform" (U[lo,hi]), "loguniform"
    (10**U[lo,hi]), "ones", or an explicit per-edge array."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    u, v = grid_edges(shape, stencil_offsets(len(shape), kind))
    if isinstance(weights, np.ndarray):
        w = weights
    elif weights == "uniform":
        w = rng.uniform(lo, hi, size=u.size)
    elif weights == "loguniform":
        w = 10.0 ** rng.uniform(lo, hi, size=u.size)
    elif weights == "ones":
        w = np.ones(u.size)
    else:
        raise ValueError(weights)
    colptr, rowind, vals = laplacian_from_edges(n, u, v, w, shift)
    return n, colptr, rowind, vals


def _haar_rotations(rng, count):
    G = rng.standard_normal((count, 3, 3))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diagonal(R, axis1=1, axis2=2))
    s[s == 0] = 1.0
    Q = Q * s[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1.0
    return Q


def elasticity_27pt(side, rng, delta=1e-2, lam_lo=1.0, lam_hi=10.0):
    """3 dofs per node on a side^3 grid with the 27-point stencil.

    For each undirected edge (u, v): K_uv = Q diag(lam) Q^T with Q a Haar
    rotation (QR of a 3x3 Gaussian, sign-fixed, det +1) and lam ~ U[1,10]^3.
    A = sum_edges (e_u - e_v)(e_u - e_v)^T (x) K_uv + delta*I.  Draw order:
    all rotations' Gaussians first, then all eigenvalue triples.
    """
    shape = (side, side, side)
    nn = side ** 3
    n = 3 * nn
    u, v = grid_edges(shape, stencil_offsets(3, "box"))
    E = u.size
    Q = _haar_rotations(rng, E)
    lam = rng.uniform(lam_lo, lam_hi, size=(E, 3))
    K = np.einsum("eij,ej,ekj->eik", Q, lam, Q)
    K = 0.5 * (K + np.transpose(K, (0, 2, 1)))
    a = np.arange(3)
    # off-diagonal blocks: rows 3v+a, cols 3u+b, value -K[a, b]
    ro = (3 * v[:, None, None] + a[None, :, None]).repeat(3, axis=2)
    co = (3 * u[:, None, None] + a[None, None, :]).repeat(3, axis=1)
    vo = -K
    # diagonal blocks: D_u += K, D_v += K
    D = np.zeros((nn, 3, 3))
    np.add.at(D, u, K)
    np.add.at(D, v, K)
    D += delta * np.eye(3)[None]
    il, jl = np.tril_indices(3)
    rd = (3 * np.arange(nn)[:, None] + il[None, :])
    cd = (3 * np.arange(nn)[:, None] + jl[None, :])
    vd = D[:, il, jl]
    rows = np.concatenate([ro.ravel(), rd.ravel()])
    cols = np.concatenate([co.ravel(), cd.ravel()])
    vals = np.concatenate([vo.ravel(), vd.ravel()])
    colptr, rowind, vv = _lower_csc(n, rows, cols, vals)
    return n, colptr, rowind, vv


def gaussian_random_field(shape, rng, ell=4.0, std=1.0, pad=2):
    """Squared-exponential-covariance Gaussian random field by FFT synthesis.

    Synthesised on a periodic lattice `pad` times larger per axis, cropped to
    `shape` and normalised to empirical mean 0 and standard deviation `std`.
    """
    big = tuple(pad * s for s in shape)
    grids = np.meshgrid(*[np.minimum(np.arange(b), b - np.arange(b)) for b in big],
                        indexing="ij")
    d2 = sum(g.astype(np.float64) ** 2 for g in grids)
    cov = np.exp(-d2 / (2.0 * ell * ell))
    S = np.maximum(np.fft.fftn(cov).real, 0.0)
    xi = rng.standard_normal(big)
    f = np.fft.ifftn(np.sqrt(S) * np.fft.fftn(xi)).real
    f = f[tuple(slice(0, s) for s in shape)]
    f = (f - f.mean()) / f.std() * std
    # array indexed [x, y, z] -> flatten with x fastest
    return np.ascontiguousarray(f.transpose(tuple(reversed(range(len(shape)))))).ravel()


def grf_laplacian(side, rng, ell=4.0, std=1.0, shift=1e-2):
    shape = (side, side, side)
    g = gaussian_random_field(shape, rng, ell=ell, std=std)
    u, v = grid_edges(shape, stencil_offsets(3, "star"))
    w = np.exp(0.5 * (g[u] + g[v]))
    n = side ** 3
    colptr, rowind, vals = laplacian_from_edges(n, u, v, w, shift)
    return n, colptr, rowind, vals, g


# --------------------------------------------------------------------------
# small random SPD matrices (tests)
# --------------------------------------------------------------------------

def random_spd(n, density, rng, dominance=1.0):
    """Random symmetric pattern, values making A strictly diagonally dominant."""
    if n == 0:
        return (0, np.zeros(1, np.int64), np.zeros(0, np.int64), np.zeros(0))
    mask = rng.random((n, n)) < density
    mask = np.tril(mask | mask.T, -1)
    r, c = np.nonzero(mask)
    w = rng.uniform(0.1, 1.0, size=r.size) * rng.choice([-1.0, 1.0], size=r.size)
    diag = np.full(n, float(dominance))
    np.add.at(diag, r, np.abs(w))
    np.add.at(diag, c, np.abs(w))
    rows = np.concatenate([r, np.arange(n)])
    cols = np.concatenate([c, np.arange(n)])
    vals = np.concatenate([w, diag])
    colptr, rowind, vv = _lower_csc(n, rows, cols, vals)
    return n, colptr, rowind, vv


def leaf_pair_spd(k, r, rng):
    """Two dense leaf blocks of k columns, not coupled to each other, each
    coupled densely to a dense parent block of r rows (ordered last): with
    the identity ordering the leaves are supernodes of k columns and k + r
    rows whose update goes to the parent.  Values strictly diagonally
    dominant."""
    n = 2 * k + r
    rows, cols = [], []
    par = np.arange(2 * k, n)
    for b in range(2):
        leaf = np.arange(b * k, (b + 1) * k)
        for j in leaf:
            below = np.concatenate([leaf[leaf > j], par])
            rows.append(below)
            cols.append(np.full(below.size, j))
    for j in par:
        below = par[par > j]
        rows.append(below)
        cols.append(np.full(below.size, j))
    r_ = np.concatenate(rows).astype(np.int64) if rows else np.zeros(0, np.int64)
    c_ = np.concatenate(cols).astype(np.int64) if cols else np.zeros(0, np.int64)
    w = rng.uniform(0.1, 1.0, size=r_.size) * rng.choice([-1.0, 1.0], size=r_.size)
    diag = np.ones(n)
    np.add.at(diag, r_, np.abs(w))
    np.add.at(diag, c_, np.abs(w))
    colptr, rowind, vv = _lower_csc(n, np.concatenate([r_, np.arange(n)]), np.concatenate([c_, np.arange(n)]),
                                    np.concatenate([w, diag]))
    return n, colptr, rowind, vv


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

CONFIG_DOC = {
    0: "2D 5-point Laplacian 32x32, w~U[0.5,1.5], shift 1e-2, ND, fundamental supernodes, 1 RHS",
    1: "3D 7-point Laplacian 64^3, w=10^U(-2,2), shift 1e-6, ND, amalgamation z=8, 1 RHS",
    2: "3D 27-point, 3 dofs, 40^3, rotated SPD 3x3 blocks (eig U[1,10]), delta 1e-2, ND, z=8, 8 RHS",
    3: "batch of 512 2D/3D grid Laplacians (2D side U{12..48}, 3D side U{8..20}), weights as cfg 0, z=8, 4 RHS",
    4: "3D 7-point Laplacian 48^3, GRF log-conductivity (ell=4, std=1), shift 1e-2, ND, "
       "greedy supernode merging (25 % cap), 1 RHS",
}

DEFAULT_AMALG = {0: 0, 1: 8, 2: 8, 3: 8, 4: 8}
DEFAULT_SNODE_MODE = {0: 0, 1: 0, 2: 0, 3: 0, 4: 0}
# amalgamation rule per workload: (0, -) the per-column zero cap amalg_z,
# (1, cap) greedy merging up to cap percent of nnz(L); the 48^3 random-field
# workload does not fix a rule, so it takes the paper's (25 %)
DEFAULT_AMALG_RULE = {0: (0, 25), 1: (0, 25), 2: (0, 25), 3: (0, 25), 4: (1, 25)}


def make_config(i: int, seed: int | None = None, side: int | None = None) -> Problem:
    """Build workload i (0, 1, 2, 4).  `side` overrides the grid side for
    reduced-size variants used by tests (same recipe, smaller grid)."""
    if seed is None:
        seed = BASE_SEED + i
    rng = np.random.default_rng(seed)
    if i == 0:
        s = side or 32
        shape = (s, s)
        n, cp, ri, vv = grid_laplacian(shape, rng, "uniform", 0.5, 1.5, 1e-2)
        perm = nested_dissection(shape)
        nrhs = 1
    elif i == 1:
        s = side or 64
        shape = (s, s, s)
        n, cp, ri, vv = grid_laplacian(shape, rng, "loguniform", -2.0, 2.0, 1e-6)
        perm = nested_dissection(shape)
        nrhs = 1
    elif i == 2:
        s = side or 40
        n, cp, ri, vv = elasticity_27pt(s, rng)
        perm = expand_block_perm(nested_dissection((s, s, s)), 3)
        nrhs = 8
    elif i == 4:
        s = side or 48
        n, cp, ri, vv, _ = grf_laplacian(s, rng)
        perm = nested_dissection((s, s, s))
        nrhs = 1
    else:
        raise ValueError("config 3 is a batch: use make_batch")
    B = rng.standard_normal((nrhs, n)).T.copy(order="F")
    meta = dict(config=i, seed=seed, side=s, amalg_z=DEFAULT_AMALG[i], amalg_rule=DEFAULT_AMALG_RULE[i][0],
                amalg_cap_percent=DEFAULT_AMALG_RULE[i][1], snode_mode=DEFAULT_SNODE_MODE[i], doc=CONFIG_DOC[i])
    return Problem(n, cp, ri, vv, perm, B, meta)


def make_batch(count: int = 512, seed: int | None = None, nrhs: int = 4,
               side2=(12, 48), side3=(8, 20)) -> list[Problem]:
    """Workload 3: `count` independent grid Laplacians of uneven sizes.

    Draw order: for each matrix, its kind (2D/3D with probability 1/2 each)
    and its integer side (inclusive range); then, matrix by matrix, the edge
    weights U[0.5, 1.5] followed by its RHS.
    """
    if seed is None:
        seed = BASE_SEED + 3
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 2, size=count)  # 0 -> 2D, 1 -> 3D
    sides = np.where(kinds == 0,
                     rng.integers(side2[0], side2[1] + 1, size=count),
                     rng.integers(side3[0], side3[1] + 1, size=count))
    out = []
    for t in range(count):
        s = int(sides[t])
        shape = (s, s) if kinds[t] == 0 else (s, s, s)
        n, cp, ri, vv = grid_laplacian(shape, rng, "uniform", 0.5, 1.5, 1e-2)
        B = rng.standard_normal((nrhs, n)).T.copy(order="F")
        perm = nested_dissection(shape)
        out.append(Problem(n, cp, ri, vv, perm, B,
                           dict(config=3, index=t, shape=shape, seed=seed, amalg_z=DEFAULT_AMALG[3],
                                snode_mode=0)))
    return out
