// HIP kernels (gfx950) for the numeric phase of right-looking supernodal
// Cholesky (Sec. II-A), the supernodal triangular solves and logdet.
//
// Every launch processes a precomputed list of independent tasks (one
// workgroup each): the supernodes of one level of the supernodal
// elimination tree (Fig. 1), split into panels of at most 64 columns and
// 64-row tiles.  Storage: supernode J is a dense column-major m_J x k_J
// array (Sec. II-A), leading dimension m_J.
#include <algorithm>
#include <climits>

#include "consts.hpp"
#include "device.hpp"

namespace spchol {

constexpr int TILE = 64;   // rows (and columns) of a tile
constexpr int NBMAX = 64;  // widest panel
constexpr int KC = 16;     // K chunk of the update GEMM

// ---------------------------------------------------------------------------
// value scatter (storage zero fill + A -> L)
// ---------------------------------------------------------------------------

__global__ void k_fill(double* __restrict__ p, int64_t count, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

__global__ void k_status_init(unsigned long long* status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *status = ULLONG_MAX;
}

// the pivot status as if column col (0-based, permuted) had failed
__global__ void k_status_min(unsigned long long* status, unsigned long long col) {
  if (threadIdx.x == 0) atomicMin(status, col);
}

__global__ void k_scatter_values(const int64_t* __restrict__ amap, const double* __restrict__ vals,
                                 int64_t nnz, double* __restrict__ L) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < nnz; i += stride) L[amap[i]] = vals[i];
}

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------

typedef double d4 __attribute__((ext_vector_type(4)));

// value of x in lane l (l uniform across the wavefront)
__device__ inline double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// panel factorization (Sec. II-A: DPOTRF then DTRSM).  The diagonal block
// of the panel lives in LDS, column-major (Dc[c * DLD + i] = D_ic).  The
// Cholesky of the block runs on one wavefront, lane = row, over 16-column
// blocks with small register micro-kernels inside rolled loops (code that
// stays in the instruction cache):
//   potrf16: right-looking sweep over the 16 columns of block b, one row per
//            lane, column j broadcast with readlane: factors D_bb on its
//            lanes and solves the rows below it on theirs
// The triangular solve of the panel's rows is a product with the inverted
// diagonal block on the matrix cores (k_panel, k_panel_rows).
// ---------------------------------------------------------------------------

constexpr int DLD = NBMAX + 2;  // even: 16-byte aligned columns
constexpr int MB = 16;          // micro-block width

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// for the inverse square root, y <- y + (y/2)(1 - x y^2) (each step doubles
// the correct bits of the estimate); a few ulps from the rounded value, on
// a much shorter dependency chain than a rounded sqrt and division.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Columns of the block past kp are padded with an identity (unit
// diagonal, zero off-diagonal), so they factor to themselves and the sweep
// needs no per-column branch.  The pivot and the entries of the scaled
// column that the other rows need (rows j0+c, c > q, one per lane) come
// straight from their lanes' registers with readlane (scalar operands of
// the row update), so the sweep never touches memory.  As in LAPACK's
// unblocked Cholesky the column is scaled by the reciprocal of the pivot's
// square root; here both come from one inverse square root,
// L_jj = d * (1/sqrt(d)).  A non-positive (or NaN) pivot is replaced by 1 so
// the sweep runs on, and the first such column is reported after it.
template <int NQ>
__device__ __forceinline__ void potrf16(double (&r)[MB], int lane, int j0, unsigned long long* __restrict__ status,
                                        int64_t col0) {
  int bad = NQ;
  // software-pipelined: the next column is updated, its pivot read and its
  // inverse square root started right after the current column is scaled;
  // the updates of the other columns fill that chain's latency
  auto pivot = [&](double d, int q, double& rinv) {
    const bool ok = d > 0.0;
    bad = (!ok && bad == NQ) ? q : bad;
    d = ok ? d : 1.0;
    rinv = rsqrt_nr(d);
    return d;
  };
  double rinv;
  double piv = pivot(readlane_d(r[0], j0), 0, rinv);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double ljj = piv * rinv;
    const double lq = (lane == j0 + q) ? ljj : (lane > j0 + q ? r[q] * rinv : 0.0);
    r[q] = lq;
    double pivn = 1.0, rinvn = 1.0;
    if (q + 1 < NQ) {
      r[q + 1] = fma(-lq, readlane_d(lq, j0 + q + 1), r[q + 1]);
      pivn = pivot(readlane_d(r[q + 1], j0 + q + 1), q + 1, rinvn);
    }
#pragma unroll
    for (int c = q + 2; c < NQ; ++c) r[c] = fma(-lq, readlane_d(lq, j0 + c), r[c]);
    piv = pivn;
    rinv = rinvn;
  }
  if (bad < NQ && lane == 0) atomicMin(status, (unsigned long long)(col0 + bad));
}

// One wavefront's share of X = A V^T for a 64-row tile (A staged in LDS
// column-major As[k * DLD + r], V column-major Wc[c * DLD + i] = V_ic):
// wavefront w computes the 16 output columns 16w..16w+15 of all 64 rows on
// the fp64 matrix cores and stores sign * X to rows R0 + r < rowEnd of dst
// (dst[c * ld + row]); with lower set only entries row >= R0 + c are stored.
// K = kp (columns past kp are zero in As).
__device__ __forceinline__ void tile_mfma_acc(const double* __restrict__ As, const double* __restrict__ Wc, int kp,
                                              int lane, int w, d4 (&acc)[4]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  // k in chunks of 16: all LDS operands of a chunk are read before its
  // 16 MFMAs
  for (int s0 = 0; s0 < kp; s0 += 16) {
    double bv[4], av[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bv[s] = Wc[(s0 + 4 * s + lk) * DLD + MB * w + li];
#pragma unroll
      for (int rb2 = 0; rb2 < 4; ++rb2) av[s][rb2] = As[(s0 + 4 * s + lk) * DLD + 16 * rb2 + li];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rb2 = 0; rb2 < 4; ++rb2)
        acc[rb2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][rb2], bv[s], acc[rb2], 0, 0, 0);
  }
}

__device__ __forceinline__ void tile_mfma(const double* __restrict__ As, const double* __restrict__ Wc, int kp,
                                          int lane, int w, double* __restrict__ dst, int ld, int R0, int rowEnd,
                                          bool lower, double sign) {
  if (MB * w >= kp) return;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[4];
  tile_mfma_acc(As, Wc, kp, lane, w, acc);
  const int c = MB * w + li;
  if (c < kp) {
    double* d = dst + (int64_t)c * ld;
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = 16 * rb2 + 4 * v + lk;
        const int r = R0 + rr;
        if (r < rowEnd && (!lower || rr >= c)) d[r] = sign * acc[rb2][v];
      }
  }
}

// stage rows R0..R0+63 of the panel (kp columns) into As, zero padded
// A value the compiler must treat as produced here (an empty asm, no
// instruction): keeps the use of a prefetched load, and the wait for it, at
// this point instead of hoisted next to the load, ahead of later loads.
__device__ __forceinline__ double here(double v) {
  asm volatile("" : "+v"(v));
  return v;
}

// A 64 x kp block of L (rows R0.. of the columns at Lp) in two steps, so
// that other loads can be issued in between: load_rows fetches thread tid's
// 16 entries (idx = u * 256 + tid, row idx & 63, column idx >> 6) from
// clamped in-bounds addresses, store_rows writes them to As (column-major,
// leading dimension DLD) with the entries past kp / m set to zero.
__device__ __forceinline__ void load_rows(double (&v)[NBMAX * NBMAX / 256], const double* __restrict__ Lp, int m,
                                          int kp, int R0, int tid) {
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx & 63, c = idx >> 6;
    v[u] = Lp[(int64_t)min(c, kp - 1) * m + min(R0 + r, m - 1)];
  }
}

__device__ __forceinline__ void store_rows(double* __restrict__ As, const double (&v)[NBMAX * NBMAX / 256], int m,
                                           int kp, int R0, int tid) {
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx & 63, c = idx >> 6;
    As[c * DLD + r] = (c < kp && R0 + r < m) ? here(v[u]) : 0.0;
  }
}

// W = inverse of the lower-triangular block in Dc (column-major, padded
// with an identity past kp; Wc zeroed beforehand), by 16 x 16 blocks:
// wavefront b inverts L_bb by substitution, then computes
// W_ib = -W_ii sum_{t=b}^{i-1} L_it W_tb on the matrix cores.
__device__ __forceinline__ void invert_diag_block(const double* __restrict__ Dc, double* __restrict__ Wc, int nblk,
                                                  int lane, int w) {
  // inverses of the 16 x 16 diagonal blocks: lane l < 16 of wavefront w
  //     computes column l of inv(L_ww)
  if (w < nblk && lane < MB) {
    const int b0 = MB * w;
    double x[MB], rd[MB];
    // the reciprocals are independent of each other (no division on the
    // substitution's dependency chain)
#pragma unroll
    for (int i = 0; i < MB; ++i) rd[i] = 1.0 / Dc[(b0 + i) * DLD + b0 + i];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < i; ++q) s = fma(-Dc[(b0 + q) * DLD + b0 + i], x[q], s);
      x[i] = s * rd[i];
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) Wc[(b0 + lane) * DLD + b0 + i] = x[i];
  }
  __syncthreads();
  // off-diagonal blocks of column block b = w, top to bottom
  if (w < nblk) {
    const int b = w, li = lane & 15, lk = lane >> 4;
    for (int i = b + 1; i < nblk; ++i) {
      d4 T = d4{0.0, 0.0, 0.0, 0.0};
      for (int tb = b; tb < i; ++tb)
#pragma unroll
        for (int s = 0; s < MB; s += 4) {
          const double av = Dc[(MB * tb + s + lk) * DLD + MB * i + li];   // L[16i + li][16tb + s + lk]
          const double bv = Wc[(MB * b + li) * DLD + MB * tb + s + lk];   // W[16tb + s + lk][16b + li]
          T = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, T, 0, 0, 0);
        }
      // W_ib = -W_ii T; T's accumulator element v is exactly the B operand
      // of k-step v (row 4v + lk, column li)
      d4 O = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double av = Wc[(MB * i + 4 * s + lk) * DLD + MB * i + li];  // W[16i + li][16i + 4s + lk]
        O = __builtin_amdgcn_mfma_f64_16x16x4f64(av, T[s], O, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Wc[(MB * b + li) * DLD + MB * i + 4 * v + lk] = -O[v];
    }
  }
}

// Panel step, diagonal part (256 threads, one task per supernode panel):
//   1. wavefront 0 factors the diagonal block in LDS (left-looking over
//      16-column blocks, potrf16 on each), writes it back, reports a
//      non-positive pivot;
//   2. W = L_pp^{-1} by 16 x 16 blocks: wavefront b inverts L_bb by
//      substitution, then W_ib = -W_ii sum_{t=b}^{i-1} L_it W_tb on the
//      matrix cores;
//   3. the next 256 rows of the panel: X = B W^T (triangular solve as a
//      product with the inverted diagonal block);
//   4. W is stored (winv) for the row-tile launch and the solves.
constexpr int PANEL_SMEM = 2 * NBMAX * DLD;  // doubles: Dc, Wc

// X = A V^T as tile_mfma_acc computes it, with A staged in LDS and V read
// from registers in the MFMA B-operand layout: bv[ks] = V[16 w + li][4 ks + lk].
__device__ __forceinline__ void tile_mfma_acc_rv(const double* __restrict__ As, const double (&bv)[NBMAX / 4], int lane,
                                                 d4 (&acc)[4]) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < NBMAX / 4; ++ks) {
    double av[4];
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2) av[rb2] = As[(4 * ks + lk) * DLD + 16 * rb2 + li];
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2) acc[rb2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb2], bv[ks], acc[rb2], 0, 0, 0);
  }
}

// One-launch panel rounds (task field c = 3, 4; 64-column panels): the
// rows of panel p's diagonal block in panel p-1's columns,
// B = L[c0 .. c0+kp, c0-64 .. c0], are solved by the diagonal task itself:
// (c = 4) B -= A2 C2^T with A2 = L[c0.., c0-128 .. c0-64] and
// C2 = L[c0-64 .., c0-128 .. c0-64] (panel p-2's update of B), then
// X = B W_{p-1}^T (W the stored inverse of panel p-1's diagonal block),
// stored in place of B.  The diagonal block, staged in Dc from v
// (identity-padded past kp), takes panel p-2's update A2 A2^T here (c = 4);
// on return Wc holds X in the layout of store_rows, for the pre-update
// D -= X X^T of c = 1 that follows.  All 256 threads; rows of X past kp
// zero.
__device__ __forceinline__ void fused_prologue(const DevSym& S, double* __restrict__ L, int J, int p, int m, int kp,
                                               bool two, const double (&v)[NBMAX * NBMAX / 256],
                                               const double* __restrict__ winv, double* __restrict__ Dc,
                                               double* __restrict__ Wc, int tid) {
  constexpr int nb = NBMAX;
  const int c0 = p * nb;
  const int lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int col = MB * w + li;  // this thread's output column (accumulator layout)
  double* __restrict__ P1 = L + S.loff[J] + (int64_t)(c0 - nb) * m;  // panel p-1's columns
  const double* __restrict__ P2 = P1 - (int64_t)nb * m;               // panel p-2's (c = 4)
  const double* __restrict__ W1 = winv + S.wbase[J] + (int64_t)(p - 1) * nb * nb;
  // every load issued together: B in the accumulator layout (rows
  // 16 rb2 + 4 q + lk, column col; rows past kp clamped, zeroed when
  // staged), W_{p-1} and C2 in the B-operand layout, A2 for LDS
  double bq[4][4], wb[NBMAX / 4], cb[NBMAX / 4], a2[NBMAX * NBMAX / 256];
#pragma unroll
  for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[rb2][q] = P1[(int64_t)col * m + c0 + min(16 * rb2 + 4 * q + lk, kp - 1)];
#pragma unroll
  for (int ks = 0; ks < NBMAX / 4; ++ks) wb[ks] = W1[(4 * ks + lk) * nb + col];
  if (two) {
#pragma unroll
    for (int ks = 0; ks < NBMAX / 4; ++ks) cb[ks] = P2[(int64_t)(4 * ks + lk) * m + c0 - nb + col];
    load_rows(a2, P2, m, nb, c0, tid);
  }
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, i = idx & 63, c = idx >> 6;
    Dc[c * DLD + i] = (i < kp && c <= i) ? here(v[u]) : (i == c ? 1.0 : 0.0);
  }
  d4 acc[4];
  if (two) {
    store_rows(Wc, a2, m, nb, c0, tid);
    __syncthreads();
    // the diagonal block less A2 A2^T (each thread its own entries)
    tile_mfma_acc(Wc, Wc, nb, lane, w, acc);
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rb2 + 4 * q + lk;
        if (r < kp && col <= r) Dc[col * DLD + r] -= acc[rb2][q];
      }
    // B less A2 C2^T
    tile_mfma_acc_rv(Wc, cb, lane, acc);
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int q = 0; q < 4; ++q) bq[rb2][q] -= acc[rb2][q];
    __syncthreads();
  }
  // X = B W^T: B (rows past kp zero) staged as the A operand
#pragma unroll
  for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rb2 + 4 * q + lk;
      Wc[col * DLD + r] = r < kp ? bq[rb2][q] : 0.0;
    }
  __syncthreads();
  tile_mfma_acc_rv(Wc, wb, lane, acc);
#pragma unroll
  for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rb2 + 4 * q + lk;
      if (r < kp) P1[(int64_t)col * m + c0 + r] = acc[rb2][q];
    }
  __syncthreads();
  // Wc <- X
#pragma unroll
  for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * rb2 + 4 * q + lk;
      Wc[col * DLD + r] = r < kp ? acc[rb2][q] : 0.0;
    }
  __syncthreads();
}

__device__ __forceinline__ void panel_body(const DevSym& S, double* __restrict__ L, const DevTask t,
                                           unsigned long long* __restrict__ status, double* __restrict__ winv,
                                           double* __restrict__ smem) {
  double* __restrict__ Dc = smem;
  double* __restrict__ Wc = smem + NBMAX * DLD;
  const int J = t.J, p = t.a, rb = t.b;
  // c = 1: panel p-1's update of the diagonal block from its solved rows;
  // c = 3, 4: those rows solved here first (one-launch rounds)
  const bool pre = t.c != 0, fused = t.c >= 3;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb;
  const int kp = min(S.nb, k - c0);
  const int nblk = (kp + MB - 1) / MB;
  double* __restrict__ Lp = L + S.loff[J] + (int64_t)c0 * m;  // Lp[c * m + r] = L[r, c0 + c]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  // the diagonal block (identity-padded past kp) and, for c = 1, rows
  // c0..c0+63 of panel p - 1 (else a dummy, never used): both loads in
  // flight together
  double v[NBMAX * NBMAX / 256], va[NBMAX * NBMAX / 256];
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, i = idx & 63, c = idx >> 6;
    v[u] = Lp[(int64_t)min(c, kp - 1) * m + c0 + min(i, kp - 1)];
  }
  if (fused) {
    fused_prologue(S, L, J, p, m, kp, t.c == 4, v, winv, Dc, Wc, tid);
  } else {
    if (pre) load_rows(va, L + S.loff[J] + (int64_t)(c0 - S.nb) * m, m, S.nb, c0, tid);
#pragma unroll
    for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
      const int idx = u * 256 + tid, i = idx & 63, c = idx >> 6;
      Dc[c * DLD + i] = (i < kp && c <= i) ? here(v[u]) : (i == c ? 1.0 : 0.0);
    }
    // (c = 1) the previous panel's rows, for the pre-update
    if (pre) store_rows(Wc, va, m, S.nb, c0, tid);
  }

  const int li = lane & 15, lk = lane >> 4;
  // wavefront 0: sweep block column b (rows >= 16b) in registers; the
  // sweep factors the 16 x 16 block (its lanes) and, on the lanes below it,
  // solves those rows against it; a block of at most 4 real columns (most
  // supernodes of the lower levels) sweeps only those, the identity-padded
  // rest is unchanged
  auto sweep = [&](int b) {
    const int j0 = MB * b, jn = min(MB, kp - j0);
    double xb[MB];
#pragma unroll
    for (int q = 0; q < MB; ++q) xb[q] = (lane >= j0) ? Dc[(j0 + q) * DLD + lane] : 0.0;
    if (jn <= 4) potrf16<4>(xb, lane, j0, status, (int64_t)S.sfirst[J] + c0 + j0);
    else potrf16<MB>(xb, lane, j0, status, (int64_t)S.sfirst[J] + c0 + j0);
    if (lane >= j0 && lane < kp) {
#pragma unroll
      for (int q = 0; q < MB; ++q)
        if (q < jn) Dc[(j0 + q) * DLD + lane] = (j0 + q <= lane) ? xb[q] : 0.0;
    }
  };
  // one wavefront, matrix cores: D(i, bp) -= L(i, jb) L(bp, jb)^T on 16 x 16
  // blocks of Dc (the whole block; above the diagonal is never read)
  auto upd_tile = [&](int i, int bp, int jb) {
    d4 P = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < MB; s += 4) {
      const double av = Dc[(MB * jb + s + lk) * DLD + MB * i + li];   // L[16i + li][16jb + s + lk]
      const double bv = Dc[(MB * jb + s + lk) * DLD + MB * bp + li];  // L[16bp + li][16jb + s + lk]
      P = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, P, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Dc[(MB * bp + li) * DLD + MB * i + 4 * v + lk] -= P[v];
  };

  if (kp == NBMAX) {
    // A full panel, pipelined: before the sweep of block b only block
    // column b has to be complete, so the rest of the work runs on
    // wavefronts 1-3 beside the sweep:
    //   step b: wavefront 0 sweeps block b; the others apply (b = 0) the
    //           previous panel's update to block columns 1-3, (b >= 1) block
    //           b-1's update to block columns b+1.., and invert diagonal
    //           block b-1 with the rest of row b-1 of W;
    //   then:   block b's update of block column b+1 (all wavefronts);
    //   last:   diagonal block 3 of W, then row 3 of W.
    // (c = 1) D -= A A^T, A = rows c0..c0+63 of panel p - 1 staged in Wc
    auto pre_tile = [&](int i, int c) {
      d4 P = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NBMAX; s += 4) {
        const double av = Wc[(s + lk) * DLD + MB * i + li];
        const double bv = Wc[(s + lk) * DLD + MB * c + li];
        P = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, P, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Dc[(MB * c + li) * DLD + MB * i + 4 * v + lk] -= P[v];
    };
    // W_bb = inverse of L_bb by substitution: lane l < 16 forms column l
    auto inv_diag = [&](int b) {
      if (lane < MB) {
        const int b0 = MB * b;
        double x[MB], rd[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) rd[i] = 1.0 / Dc[(b0 + i) * DLD + b0 + i];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          double z = (i == lane) ? 1.0 : 0.0;
#pragma unroll
          for (int q = 0; q < i; ++q) z = fma(-Dc[(b0 + q) * DLD + b0 + i], x[q], z);
          x[i] = z * rd[i];
        }
#pragma unroll
        for (int i = 0; i < MB; ++i) Wc[(b0 + lane) * DLD + b0 + i] = x[i];
      }
    };
    // W_ib = -W_ii sum_{t=b}^{i-1} L_it W_tb (W_tb and W_ii already formed)
    auto inv_off = [&](int i, int b) {
      d4 T = d4{0.0, 0.0, 0.0, 0.0};
      for (int tb = b; tb < i; ++tb)
#pragma unroll
        for (int s = 0; s < MB; s += 4) {
          const double av = Dc[(MB * tb + s + lk) * DLD + MB * i + li];  // L[16i + li][16tb + s + lk]
          const double bv = Wc[(MB * b + li) * DLD + MB * tb + s + lk];  // W[16tb + s + lk][16b + li]
          T = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, T, 0, 0, 0);
        }
      // T's accumulator element v is exactly the B operand of k-step v
      d4 O = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double av = Wc[(MB * i + 4 * s + lk) * DLD + MB * i + li];  // W[16i + li][16i + 4s + lk]
        O = __builtin_amdgcn_mfma_f64_16x16x4f64(av, T[s], O, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Wc[(MB * b + li) * DLD + MB * i + 4 * v + lk] = -O[v];
    };
    if (pre) {
      __syncthreads();
      pre_tile(w, 0);  // block column 0, one block per wavefront
    }
    __syncthreads();
    for (int b = 0; b < 4; ++b) {
      if (w == 0) {
        sweep(b);
      } else if (b == 0) {
        // the previous panel's update of block columns 1-3, two blocks per
        // wavefront: (1,1) (2,1) | (3,1) (2,2) | (3,2) (3,3)
        if (pre) {
          if (w == 1) { pre_tile(1, 1); pre_tile(2, 1); }
          else if (w == 2) { pre_tile(3, 1); pre_tile(2, 2); }
          else { pre_tile(3, 2); pre_tile(3, 3); }
        }
      } else if (w == 1) {
        inv_diag(b - 1);
        for (int j = b - 2; j >= 0; --j) inv_off(b - 1, j);
      } else if (b == 1) {
        // block 0's update of block columns 2-3: (2,2) (3,3) | (3,2)
        if (w == 2) { upd_tile(2, 2, 0); upd_tile(3, 3, 0); }
        else upd_tile(3, 2, 0);
      } else if (b == 2 && w == 2) {
        upd_tile(3, 3, 1);  // block 1's update of block column 3
      }
      __syncthreads();
      if (b < 3) {
        // Wc is free once the previous panel's update is applied: cleared
        // for W, whose blocks above the diagonal stay zero
        if (b == 0)
          for (int idx = tid; idx < NBMAX * DLD; idx += 256) Wc[idx] = 0.0;
        if (w <= 2 - b) upd_tile(b + 1 + w, b + 1, b);  // block column b+1 by block b
        __syncthreads();
      }
    }
    // write the factored block back (lower part), all threads, coalesced
#pragma unroll
    for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
      const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
      if (c <= r) Lp[(int64_t)c * m + c0 + r] = Dc[c * DLD + r];
    }
    if (w == 0) inv_diag(3);
    __syncthreads();
    if (w < 3) inv_off(3, w);
    __syncthreads();
  } else {
    // 0. (c = 1) the previous panel's update of the diagonal block,
    //    D -= A A^T with A = rows c0..c0+kp of panel p - 1, on the matrix
    //    cores (A staged in Wc, which is cleared again afterwards)
    if (pre) {
      __syncthreads();
      d4 acc[4];
      tile_mfma_acc(Wc, Wc, S.nb, lane, w, acc);
      const int c = MB * w + (lane & 15), lk = lane >> 4;
#pragma unroll
      for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * rb2 + 4 * q + lk;
          if (r < kp && c <= r) Dc[c * DLD + r] -= acc[rb2][q];
        }
      // a last, narrower panel: rows kp..63 of the tile lie below its
      // diagonal block, in storage (the row-tile launch reads them next;
      // in one-launch rounds the row tiles apply this update themselves)
      if (kp < NBMAX && !fused) {
#pragma unroll
        for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = 16 * rb2 + 4 * q + lk;
            if (r >= kp && c < kp && c0 + r < m) Lp[(int64_t)c * m + c0 + r] -= acc[rb2][q];
          }
      }
      __syncthreads();
    }
    for (int idx = tid; idx < NBMAX * DLD; idx += 256) Wc[idx] = 0.0;
    __syncthreads();

    // 1. Cholesky of the diagonal block, right-looking over 16-column blocks:
    //    wavefront 0 sweeps block column b (rows >= 16b), then the four
    //    wavefronts apply its update to the 16 x 16 blocks (i, b') with
    //    i >= b' > b on the matrix cores:
    //    D[i][b'] -= L[i][b] L[b'][b]^T
    for (int b = 0; b < nblk; ++b) {
      if (w == 0) sweep(b);
      __syncthreads();
      const int nrest = nblk - 1 - b;  // block columns right of b
      const int npairs = nrest * (nrest + 1) / 2;
      for (int pr = w; pr < npairs; pr += 4) {
        // pair index -> (i, bp) with b < bp <= i < nblk
        int bp = b + 1, rem = pr;
        while (rem >= nblk - bp) { rem -= nblk - bp; ++bp; }
        upd_tile(bp + rem, bp, b);
      }
      __syncthreads();
    }
    // write the factored block back (lower part), all threads, coalesced
#pragma unroll
    for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
      const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
      if (r < kp && c <= r) Lp[(int64_t)c * m + c0 + r] = Dc[c * DLD + r];
    }

    // 2. W = L_pp^{-1}
    invert_diag_block(Dc, Wc, nblk, lane, w);
    __syncthreads();
  }

  // 4. W, kp x kp column-major (zeros above the diagonal), for the row-tile
  //    launch and the solves
  {
    double* dst = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;
#pragma unroll
    for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
      const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
      if (r < kp && c < kp) dst[c * kp + r] = r >= c ? Wc[c * DLD + r] : 0.0;
    }
  }
  // 3. rows rb .. rb + 255, the next 64-row tile fetched while this one is
  //    solved
  {
    const int re = min(rb + 4 * 64, m);
    double vr[NBMAX * NBMAX / 256];
    if (rb < re) load_rows(vr, Lp, m, kp, rb, tid);
    for (int R0 = rb; R0 < re; R0 += 64) {
      store_rows(Dc, vr, m, kp, R0, tid);
      __syncthreads();
      if (R0 + 64 < re) load_rows(vr, Lp, m, kp, R0 + 64, tid);
      tile_mfma(Dc, Wc, kp, lane, w, Lp, m, R0, m, false, 1.0);
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_panel(DevSym S, double* __restrict__ L, int64_t off,
                                               unsigned long long* __restrict__ status,
                                               double* __restrict__ winv) {
  __shared__ __attribute__((aligned(16))) double smem[PANEL_SMEM];
  panel_body(S, L, S.tasks[off + blockIdx.x], status, winv, smem);
}

// Panel step, row tiles not solved by the diagonal task: X = B W^T with the
// inverted diagonal block W the diagonal task stored (256 threads, one
// 64-row tile each).  c = 1 (one-launch rounds): the tile first takes panel
// p-1's update, B -= A C^T with A its rows of panel p-1 and C the rows of
// panel p's diagonal block in panel p-1's columns (solved a round before).
__device__ __forceinline__ void rows_body(const DevSym& S, double* __restrict__ L, const DevTask t,
                                          const double* __restrict__ winv, double* __restrict__ smem) {
  double* __restrict__ As = smem;
  double* __restrict__ Wc = smem + NBMAX * DLD;
  const int J = t.J, p = t.a, R0 = t.b;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb;
  const int kp = min(S.nb, k - c0);
  double* __restrict__ Lp = L + S.loff[J] + (int64_t)c0 * m;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
  const double* __restrict__ src = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;
  // the inverse block and the tile's rows: both loads in flight together
  double v[NBMAX * NBMAX / 256], vr[NBMAX * NBMAX / 256];
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;  // idx = c * 64 + r
    v[u] = src[min(c, kp - 1) * kp + min(r, kp - 1)];
  }
  if (t.c == 1) {
    // B in the accumulator layout of tile_mfma_acc (wavefront w: column
    // 16 w + li, rows 16 rb2 + 4 q + lk of the tile), A and C of panel p-1
    const double* __restrict__ P1 = Lp - (int64_t)S.nb * m;
    double bq[4][4], ca[NBMAX * NBMAX / 256];
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rb2 + 4 * q + lk;
        bq[rb2][q] = Lp[(int64_t)min(MB * w + li, kp - 1) * m + min(R0 + r, m - 1)];
      }
    load_rows(vr, P1, m, S.nb, R0, tid);
    load_rows(ca, P1, m, S.nb, c0, tid);
    store_rows(As, vr, m, S.nb, R0, tid);
    store_rows(Wc, ca, m, S.nb, c0, tid);
    __syncthreads();
    d4 acc[4];
    tile_mfma_acc(As, Wc, S.nb, lane, w, acc);
    __syncthreads();
    const int c = MB * w + li;
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rb2 + 4 * q + lk;
        As[c * DLD + r] = (c < kp && R0 + r < m) ? bq[rb2][q] - acc[rb2][q] : 0.0;
      }
  } else {
    load_rows(vr, Lp, m, kp, R0, tid);
  }
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
    Wc[c * DLD + r] = (r < kp && c < kp) ? here(v[u]) : 0.0;
  }
  if (t.c != 1) store_rows(As, vr, m, kp, R0, tid);
  __syncthreads();
  tile_mfma(As, Wc, kp, lane, w, Lp, m, R0, m, false, 1.0);
}

__global__ __launch_bounds__(256) void k_panel_rows(DevSym S, double* __restrict__ L, int64_t off,
                                                    const double* __restrict__ winv) {
  __shared__ __attribute__((aligned(16))) double smem[2 * NBMAX * DLD];
  rows_body(S, L, S.tasks[off + blockIdx.x], winv, smem);
}

// ---------------------------------------------------------------------------
// update: C[i, c] -= sum_t L[i, t] L[c, t] over a 64 x 64 tile, lower part,
// on the matrix cores (16x16x4 MFMA, four wavefronts of 32 x 32, K in
// chunks of 32 staged through LDS with the next chunk prefetched into
// registers).
//   kind 1 (internal): the remaining columns of J itself, K = one panel;
//                      plain read-modify-write (one writer per entry).
//   kind 2 (external): the update matrix L_RJ L_RJ^T (Sec. II-A, Fig. 2),
//                      K = all columns of J, scattered into the ancestors
//                      through the relative indices; atomic adds because
//                      several supernodes of a level may hit one ancestor.
// Precision P: 0 = fp64 operands and accumulation; 1 = operands rounded to
// fp32 while staging into LDS, fp32 accumulation; 2 = operands rounded to
// bf16, fp32 accumulation on the 16x16x16 bf16 MFMA (the mixed-precision
// forms); the scatter is always fp64.
// MFMA operand layout (one wavefront, 16x16x4, checked on gfx950): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; fp64 accumulator
// element v holds D[4 v + l / 16][l % 16], fp32 element v holds
// D[4 (l / 16) + v][l % 16].
// ---------------------------------------------------------------------------

typedef float f4 __attribute__((ext_vector_type(4)));

template <int P> struct UpdPrec;
template <> struct UpdPrec<0> {
  using T = double;
  using Acc = d4;
  static __device__ __forceinline__ Acc zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * v + lk; }
};
template <> struct UpdPrec<1> {
  using T = float;
  using Acc = f4;
  static __device__ __forceinline__ Acc zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};
// bf16 operands, fp32 accumulation: one 16x16x16 MFMA per K chunk of 16;
// staged row-major, four consecutive k of a row packed in 8 bytes
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
// two groups of four bf16 as the eight-value operand of the double-K MFMA
__device__ __forceinline__ bf8 pair_bf8(s4 lo, s4 hi) {
  struct Two { s4 lo, hi; };
  return __builtin_bit_cast(bf8, Two{lo, hi});
}
template <> struct UpdPrec<2> {
  using T = s4;
  using Acc = f4;
  static __device__ __forceinline__ Acc zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ int row(int v, int lk) { return 4 * lk + v; }
};

// fp64 -> bf16, round to nearest even (through fp32; finite inputs)
__device__ __forceinline__ unsigned short to_bf16(double x) {
  unsigned u = __float_as_uint((float)x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

constexpr int ALD = TILE + 2;
constexpr int UKC = 32;  // K chunk of the update GEMM
constexpr int G2 = UKC / 4 + 1;  // bf16 staging: 8-byte groups per row (UKC / 4 used, 1 pad)
constexpr int CLD = TILE + 1;  // column stride of the epilogue tile

// LDS of an update tile: the operand chunks As, Bs (UKC x ALD doubles each;
// fp32 and bf16 use part of their slot) during the K loop, then the
// epilogue tile Cs (TILE x CLD doubles) in the same space.
constexpr int UPD_SMEM = (2 * UKC * ALD > TILE * CLD) ? 2 * UKC * ALD : TILE * CLD;
static_assert(TILE * G2 * sizeof(s4) <= UKC * ALD * sizeof(double), "bf16 staging fits the operand area");

template <int P, int kind>
__device__ __forceinline__ void update_body(const DevSym& S, double* __restrict__ L, const DevTask t,
                                            double* __restrict__ smem, double* __restrict__ aux = nullptr) {
  using Pr = UpdPrec<P>;
  using T = typename Pr::T;
  double* __restrict__ Cs = smem;
  T* __restrict__ As = reinterpret_cast<T*>(smem);
  T* __restrict__ Bs = reinterpret_cast<T*>(smem + UKC * ALD);
  const int J = t.J;
  const int m = S.sm[J], k = S.sk[J];
  int kb, ke, colEnd, row0 = t.a, col0 = t.b, rowEnd = m;
  if constexpr (kind == 1) {
    kb = t.c * S.nb;
    ke = min(k, kb + S.nb);
    colEnd = k;
  } else if constexpr (kind == 6) {
    // panels (c & 0xffff) .. + ((c >> 16) & 0xff) - 1
    kb = (t.c & 0xffff) * S.nb;
    ke = min(k, kb + ((t.c >> 16) & 0xff) * S.nb);
    colEnd = k;
  } else if constexpr (kind == 4) {
    // a block-pair tile: rows row0 .. rowEnd - 1, columns col0 .. colEnd - 1
    kb = 0;
    ke = k;
    row0 = t.a & ((1 << 25) - 1);
    rowEnd = row0 + (t.a >> 25) + 1;
    col0 = t.b & ((1 << 25) - 1);
    colEnd = col0 + (t.b >> 25) + 1;
  } else {
    kb = 0;
    ke = k;
    colEnd = m;
  }
  double* __restrict__ Lj = L + S.loff[J];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  typename Pr::Acc acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Pr::zero();

  // staging: thread loads rows (tid & 63) of chunk columns (tid >> 6) + 4q
  // (bf16: columns 8 (tid >> 6) + q, packed into two 8-byte groups)
  const int sr = tid & 63, sc = tid >> 6;
  const bool va = row0 + sr < rowEnd, vb = col0 + sr < colEnd;
  const double* pa = Lj + row0 + sr;
  const double* pb = Lj + col0 + sr;
  double ra[UKC / 4], rb[UKC / 4];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int q = 0; q < UKC / 4; ++q) {
      const int gc = P == 2 ? kk + (UKC / 4) * sc + q : kk + sc + 4 * q;
      ra[q] = (va && gc < ke) ? pa[(int64_t)gc * m] : 0.0;
      rb[q] = (vb && gc < ke) ? pb[(int64_t)gc * m] : 0.0;
    }
  };
  fetch(kb);
  // (external) lane l fetches tile column l's ancestor data (its pair's
  // first row and relind offset, the column's storage offset) before the
  // product, so that the scatter's row positions need one round trip after it
  // (internal) the tile's entries of the target, read now (no other task of
  // the launch touches them) so that the epilogue only stores: thread
  // (lane, w) owns row row0 + lane of columns col0 + w + 4j (clamped
  // in-bounds addresses; the values are used only where the entry exists)
  double cold[TILE / 4];
  if constexpr (kind == 1) {
    const int rr = min(row0 + lane, m - 1);
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) cold[j] = Lj[(int64_t)min(col0 + w + 4 * j, colEnd - 1) * m + rr];
  }
  int64_t cbase_l = 0, rel_l = 0;
  int a0_l = 0;
  if constexpr (kind == 4) {
    // RLB: every column of the tile lies in one ancestor P, at consecutive
    // columns of it; lane l holds the storage offset of tile column l
    const int32_t* R = S.rows + S.rptr[J];
    const int anc = S.snode_of[R[col0]];
    cbase_l = S.loff[anc] + (int64_t)(R[min(col0 + lane, colEnd - 1)] - S.sfirst[anc]) * S.sm[anc];
  } else if constexpr (kind == 2 || kind == 3) {
    const int64_t ob = S.obase[J];
    const int lc = min(col0 + lane, colEnd - 1) - k;
    const int pair_l = S.opair[ob + lc];
    cbase_l = S.ocbase[ob + lc];
    a0_l = S.pa0[pair_l];
    rel_l = S.relptr[pair_l];
  }
  if constexpr (P == 2) {
    for (int kk = kb; kk < ke; kk += UKC) {
#pragma unroll
      for (int g = 0; g < UKC / 16; ++g) {
        As[sr * G2 + (UKC / 16) * sc + g] = s4{(short)to_bf16(ra[4 * g]), (short)to_bf16(ra[4 * g + 1]),
                                                (short)to_bf16(ra[4 * g + 2]), (short)to_bf16(ra[4 * g + 3])};
        Bs[sr * G2 + (UKC / 16) * sc + g] = s4{(short)to_bf16(rb[4 * g]), (short)to_bf16(rb[4 * g + 1]),
                                                (short)to_bf16(rb[4 * g + 2]), (short)to_bf16(rb[4 * g + 3])};
      }
      __syncthreads();
      if (kk + UKC < ke) fetch(kk + UKC);
      // gfx950's double-K MFMA (16 x 16 x 32): lane (li, lk) gives eight
      // values of row li, here groups lk and 4 + lk (k = 4 lk .. + 3 and
      // 16 + 4 lk .. + 3); A and B take the same k from each lane, so the
      // product sums all 32 k whichever order the unit assigns them
      static_assert(UKC == 32, "one double-K MFMA per chunk");
      {
        const bf8 a0 = pair_bf8(As[(wr + li) * G2 + lk], As[(wr + li) * G2 + 4 + lk]);
        const bf8 a1 = pair_bf8(As[(wr + 16 + li) * G2 + lk], As[(wr + 16 + li) * G2 + 4 + lk]);
        const bf8 b0 = pair_bf8(Bs[(wc + li) * G2 + lk], Bs[(wc + li) * G2 + 4 + lk]);
        const bf8 b1 = pair_bf8(Bs[(wc + 16 + li) * G2 + lk], Bs[(wc + 16 + li) * G2 + 4 + lk]);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();
    }
  } else
  for (int kk = kb; kk < ke; kk += UKC) {
#pragma unroll
    for (int q = 0; q < UKC / 4; ++q) {
      As[(sc + 4 * q) * ALD + sr] = (T)ra[q];
      Bs[(sc + 4 * q) * ALD + sr] = (T)rb[q];
    }
    __syncthreads();
    if (kk + UKC < ke) fetch(kk + UKC);
#pragma unroll
    for (int ks = 0; ks < UKC; ks += 4) {
      const int kr = (ks + lk) * ALD;
      const T a0 = As[kr + wr + li], a1 = As[kr + wr + 16 + li];
      const T b0 = Bs[kr + wc + li], b1 = Bs[kr + wc + 16 + li];
      acc[0][0] = Pr::mma(a0, b0, acc[0][0]);
      acc[0][1] = Pr::mma(a0, b1, acc[0][1]);
      acc[1][0] = Pr::mma(a1, b0, acc[1][0]);
      acc[1][1] = Pr::mma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }

  // (external) the row positions of the lane's row in the ancestors of the
  // wavefront's 16 columns w, w + 4, ..., all loads issued before the tile
  // goes through LDS (from a clamped in-bounds index: a position is used
  // only for an entry on or below the diagonal, whose row then lies in the
  // column's ancestor)
  int tpvs[TILE / 4];
  if constexpr (kind == 4) {
    // the rows are consecutive in the ancestor too: one relative index (the
    // position of the tile's first row, task field c) for all of them
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) tpvs[j] = t.c + lane;
  } else if constexpr (kind == 2 || kind == 3) {
    const int gr = row0 + lane;
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) {
      const int cc = w + 4 * j;
      const int a0 = __builtin_amdgcn_readlane(a0_l, cc);
      const int64_t rel = ((int64_t)__builtin_amdgcn_readlane((int)(rel_l >> 32), cc) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rel_l, cc);
      const bool ok = gr < m && gr - k >= a0;
      tpvs[j] = S.tpos[ok ? rel + (gr - k - a0) : rel];
    }
  }
  // Epilogue: the tile goes through LDS so that each wavefront then owns
  // whole tile columns, one row per lane: the target addresses of a column
  // are row runs of the ancestor's storage, so the read-modify-writes (and
  // the atomics) are coalesced instead of touching 16 columns per access.
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Cs[(wc + 16 * bj + li) * CLD + wr + 16 * bi + Pr::row(v, lk)] = (double)acc[bi][bj][v];
  __syncthreads();
  const int gr = row0 + lane;
  const int cmax = min(TILE, colEnd - col0);
  if constexpr (kind == 1) {
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) {
      const int cc = w + 4 * j, gc = col0 + cc;
      if (cc < cmax && gr < m && gr >= gc) Lj[(int64_t)gc * m + gr] = cold[j] - Cs[cc * CLD + lane];
    }
  } else if constexpr (kind == 6) {
    // (other tasks of the launch add into the same entries: the other
    // panel ranges of the block)
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) {
      const int cc = w + 4 * j, gc = col0 + cc;
      if (cc < cmax && gr < m && gr >= gc) atomicAdd(Lj + (int64_t)gc * m + gr, -Cs[cc * CLD + lane]);
    }
  } else if constexpr (kind == 5) {
    // the update matrix itself, not scattered: rows cb .. m - 1 of its
    // columns cb .. (a column block, cb = task field c) go to aux,
    // column-major with leading dimension m - cb, lower part
    const int cb = t.c;
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) {
      const int cc = w + 4 * j, gc = col0 + cc;
      if (cc < cmax && gr < m && gr >= gc) aux[(int64_t)(gr - cb) + (int64_t)(gc - cb) * (m - cb)] = Cs[cc * CLD + lane];
    }
  } else {
    // target of entry (gr, gc): the ancestor column of row gc at storage
    // offset ocbase, row position tpos[relptr[pair] + gr - k - pa0[pair]]
    // with pair = (J, ancestor), fetched above
    const bool rowok = gr < rowEnd;
    // the wavefront's 16 values of the lane's row, all read before the first
    // atomic (one LDS wait, not one per column)
    double cv[TILE / 4];
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) cv[j] = Cs[(w + 4 * j) * CLD + lane];
#pragma unroll
    for (int j = 0; j < TILE / 4; ++j) cv[j] = here(cv[j]);
    if constexpr (kind == 2 || kind == 4) {
#pragma unroll
      for (int j = 0; j < TILE / 4; ++j) {
        const int cc = w + 4 * j;
        if (cc < cmax) {
          const int gc = col0 + cc;
          const int64_t cbase = ((int64_t)__builtin_amdgcn_readlane((int)(cbase_l >> 32), cc) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)cbase_l, cc);
          if (rowok && gr >= gc) atomicAdd(L + cbase + tpvs[j], -cv[j]);
        }
      }
    } else {
      // kind 3: no other task of the launch adds into these entries (the
      // launch holds supernodes with disjoint row lists), so a plain
      // read-modify-write: every read issued first (clamped to the column's
      // own storage where the entry does not exist), then the writes
      int64_t addr[TILE / 4];
      double old[TILE / 4];
#pragma unroll
      for (int j = 0; j < TILE / 4; ++j) {
        const int cc = min(w + 4 * j, cmax - 1);
        const int64_t cbase = ((int64_t)__builtin_amdgcn_readlane((int)(cbase_l >> 32), cc) << 32) |
                              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)cbase_l, cc);
        addr[j] = cbase + tpvs[j];
        old[j] = L[addr[j]];
      }
#pragma unroll
      for (int j = 0; j < TILE / 4; ++j) {
        const int cc = w + 4 * j;
        if (cc < cmax && rowok && gr >= col0 + cc) L[addr[j]] = old[j] - cv[j];
      }
    }
  }
}

// kind 1: internal update tiles, kind 2: external (scattered) update tiles.
// Four workgroups per compute unit (at most 128 registers a lane): while
// some apply their scatter, the others keep the matrix cores busy.
// Workgroup b of a launch runs on XCD b % 8 (round-robin dispatch).  With
// grp > 0 the XCDs take the task list in chunks of grp consecutive tasks
// (chunk c on XCD c % 8), so the tiles of one supernode, which read the same
// panel rows, mostly share one XCD's L2; the tail past the last whole round
// of 8 chunks keeps the plain order.  A bijection of [0, n).
__device__ __forceinline__ int32_t xcd_task(int32_t b, int32_t n, int32_t grp) {
  if (grp <= 0) return b;
  const int32_t full = n / (8 * grp) * (8 * grp);
  if (b >= full) return b;
  const int32_t x = b & 7, j = b >> 3;
  return ((j / grp) * 8 + x) * grp + j % grp;
}

template <int P, int kind>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_update(DevSym S, double* __restrict__ L,
                                                                                          int64_t off, double* aux,
                                                                                          int32_t grp) {
  __shared__ __attribute__((aligned(16))) double smem[UPD_SMEM];
  update_body<P, kind>(S, L, S.tasks[off + xcd_task((int32_t)blockIdx.x, (int32_t)gridDim.x, grp)], smem, aux);
}

// One-panel lookahead: workgroups below nfirst factor panel p (panel_body),
// the others apply internal update tiles of panel p-1 to columns right of
// panel p.  The two sets touch disjoint columns.
// One-launch panel rounds: workgroups below nfirst are diagonal tasks,
// those below ntrsm_end row tiles (rows_body), the rest internal update
// tiles; the sets touch disjoint entries.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_panel_la(DevSym S, double* __restrict__ L, int64_t off, int32_t nfirst,
                                                  int32_t ntrsm_end, unsigned long long* __restrict__ status,
                                                  double* __restrict__ winv) {
  __shared__ __attribute__((aligned(16))) double smem[PANEL_SMEM > UPD_SMEM ? PANEL_SMEM : UPD_SMEM];
  const DevTask t = S.tasks[off + blockIdx.x];
  if ((int)blockIdx.x < nfirst) panel_body(S, L, t, status, winv, smem);
  else if ((int)blockIdx.x < ntrsm_end) rows_body(S, L, t, winv, smem);
  else if (t.c & kPanelRange) update_body<P, 6>(S, L, t, smem);
  else update_body<P, 1>(S, L, t, smem);
}

// ---------------------------------------------------------------------------
// Small supernodes (at most 16 columns, the whole step within one
// wavefront): one wavefront does a supernode's entire numeric step in
// registers, one row per lane -- the Cholesky of the diagonal block, the
// solve of the rows below (Sec. II), the inverse block the solves use, and
// the update L_R L_R^T of the rows below, scattered into the ancestors
// through the relative indices (Sec. II-A).  With the swept block padded to
// NQ = 4 or 16 columns and r = m - K rows below, the lanes hold
//   0 .. K-1            the rows of the diagonal block,
//   K .. NQ-1           identity rows (the padding columns factor to
//                       themselves),
//   NQ .. NQ+r-1        the rows below,
//   NQ+r .. NQ+r+K-1    unit rows e_j: the sweep solves x L^T = e_j, so the
//                       lane ends with column j of W = L^-1 (zero above j).
// The sweep is the panel kernel's, which factors the block and solves every
// lane below it against it.  Four supernodes per workgroup, no LDS and no
// barriers.  Precision P as for the tiled updates: the update's operands
// rounded to fp32 (1) or bf16 (2) with fp32 accumulation; the diagonal
// block, the solve and the scatter are fp64.
// ---------------------------------------------------------------------------

template <int P>
__device__ __forceinline__ float low_precision(double v) {
  if constexpr (P == 2) return __uint_as_float((unsigned)to_bf16(v) << 16);
  else return (float)v;
}

template <int P>
__global__ __launch_bounds__(256) void k_small(DevSym S, double* __restrict__ L, int64_t off, int32_t ntasks,
                                               unsigned long long* __restrict__ status,
                                               double* __restrict__ winv) {
  const int lane = threadIdx.x & 63;
  const int q = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (q >= ntasks) return;  // a whole wavefront; nothing below synchronizes
  const DevTask t = S.tasks[off + q];
  const int J = t.J, m = S.sm[J], k = S.sk[J];
  const int nq = k <= 4 ? 4 : MB;
  const int r = m - k;
  const bool diag = lane < k;
  const bool below = lane >= nq && lane < nq + r;
  const bool unit = lane >= nq + r && lane < nq + r + k;
  const int row = diag ? lane : (below ? k + lane - nq : 0);         // local row of J (else 0)
  const int e = unit ? lane - nq - r : ((lane >= k && lane < nq) ? lane : -1);  // unit row
  double* __restrict__ Lj = L + S.loff[J];
  double x[MB];
#pragma unroll
  for (int c = 0; c < MB; ++c) {
    const double v = Lj[(int64_t)min(c, k - 1) * m + row];
    x[c] = ((diag || below) && c < k) ? v : (c == e ? 1.0 : 0.0);
  }
  if (nq == 4) potrf16<4>(x, lane, 0, status, (int64_t)S.sfirst[J]);
  else potrf16<MB>(x, lane, 0, status, (int64_t)S.sfirst[J]);
  if (diag || below) {
#pragma unroll
    for (int c = 0; c < MB; ++c)
      if (c < k && c <= row) Lj[(int64_t)c * m + row] = x[c];
  }
  if (unit) {
    double* __restrict__ Wd = winv + S.wbase[J];  // the one panel: K x K, column-major
#pragma unroll
    for (int c = 0; c < MB; ++c)
      if (c < k) Wd[(int64_t)e * k + c] = c >= e ? x[c] : 0.0;
  }
  if (r == 0) return;
  // update column b (local row k + b of J, a column of an ancestor): lane
  // NQ + a adds -(L_R L_R^T)_ab, a >= b, at its row's position in that
  // column; column data fetched per lane up front, row positions reloaded
  // only when the ancestor changes (as in the tiled external update)
  const int64_t ob = S.obase[J];
  const int bl = min(lane, r - 1);
  const int pair_l = S.opair[ob + bl];
  const int64_t cbase_l = S.ocbase[ob + bl];
  const int a = lane - nq;
  float xl[MB];
  if constexpr (P != 0) {
#pragma unroll
    for (int c = 0; c < MB; ++c) xl[c] = low_precision<P>(x[c]);
  }
  int cur = -1, tpv = 0;
  for (int b = 0; b < r; ++b) {
    double u;
    if constexpr (P == 0) {
      u = 0.0;
#pragma unroll
      for (int c = 0; c < MB; ++c)
        if (c < k) u = fma(x[c], readlane_d(x[c], nq + b), u);
    } else {
      float uf = 0.f;
#pragma unroll
      for (int c = 0; c < MB; ++c)
        if (c < k) uf = fmaf(xl[c], __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xl[c]), nq + b)), uf);
      u = (double)uf;
    }
    const int pair = __builtin_amdgcn_readlane(pair_l, b);
    const int64_t cbase = ((int64_t)__builtin_amdgcn_readlane((int)(cbase_l >> 32), b) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)cbase_l, b);
    if (pair != cur) {
      cur = pair;
      const int a0 = S.pa0[pair];
      tpv = (below && a >= a0) ? S.tpos[S.relptr[pair] + a - a0] : 0;
    }
    if (below && a >= b) atomicAdd(L + cbase + tpv, -u);
  }
}

// One wavefront per one-panel supernode of at most 16 (NB = 1) or 32
// (NB = 2) columns that is too tall for k_small (Sec. II: the diagonal
// block's Cholesky factor and the panel solve, here without the update,
// which the external update tiles do).  The sweep takes, as in k_small, the
// block padded to 4, 16 or 32 columns, the rows below that still fit and k
// unit rows: those come out as rows of L_JJ^{-T} (stored as the inverse
// block W = L_JJ^{-1}).  With two 16-column blocks the second is first
// updated by the first (lane broadcasts), then swept.  The remaining rows
// below follow 64 at a time, each row a times L_JJ^{-T} (a L_JJ^{-T} L_JJ^T
// = a), the entries of L_JJ^{-T} broadcast from the unit lanes, in place
// from the last column down (column c takes entries 0..c of the row).
template <int NB>
__global__ __launch_bounds__(256) void k_medium(DevSym S, double* __restrict__ L, int64_t off, int32_t ntasks,
                                                unsigned long long* __restrict__ status,
                                                double* __restrict__ winv) {
  constexpr int NC = NB * MB;
  const int lane = threadIdx.x & 63;
  const int q = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (q >= ntasks) return;  // a whole wavefront; nothing below synchronizes
  const DevTask t = S.tasks[off + q];
  const int J = t.J, m = S.sm[J], k = S.sk[J];
  const int nq = NB == 2 ? NC : (k <= 4 ? 4 : MB);
  const int r = m - k;
  const int r0 = max(0, min(r, 64 - nq - k));  // rows below inside the sweep
  const bool diag = lane < k;
  const bool below = lane >= nq && lane < nq + r0;
  const bool unit = lane >= nq + r0 && lane < nq + r0 + k;
  const int row = diag ? lane : (below ? k + lane - nq : 0);
  const int e = unit ? lane - nq - r0 : ((lane >= k && lane < nq) ? lane : -1);
  const int64_t col0 = S.sfirst[J];
  double* __restrict__ Lj = L + S.loff[J];
  double x[NB][MB];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int cc = 0; cc < MB; ++cc) {
      const int c = b * MB + cc;
      const double v = Lj[(int64_t)min(c, k - 1) * m + row];
      x[b][cc] = ((diag || below) && c < k) ? v : (c == e ? 1.0 : 0.0);
    }
  if (NB == 1 && nq == 4) potrf16<4>(x[0], lane, 0, status, col0);
  else potrf16<MB>(x[0], lane, 0, status, col0);
  if constexpr (NB == 2) {
#pragma unroll
    for (int c = 0; c < MB; ++c)
#pragma unroll
      for (int j = 0; j < MB; ++j) x[1][j] = fma(-x[0][c], readlane_d(x[0][c], MB + j), x[1][j]);
    potrf16<MB>(x[1], lane, MB, status, col0 + MB);
  }
  if (diag || below) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int cc = 0; cc < MB; ++cc) {
        const int c = b * MB + cc;
        if (c < k && c <= row) Lj[(int64_t)c * m + row] = x[b][cc];
      }
  }
  if (unit) {
    double* __restrict__ Wd = winv + S.wbase[J];  // the one panel: K x K, column-major
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int cc = 0; cc < MB; ++cc) {
        const int c = b * MB + cc;
        if (c < k) Wd[(int64_t)e * k + c] = c >= e ? x[b][cc] : 0.0;
      }
  }
  const int ub = nq + r0;  // lane of unit row 0: row u of L_JJ^{-T} in lane ub + u (u < k)
  for (int base = k + r0; base < m; base += 64) {
    const int rr = base + lane;
    const bool ok = rr < m;
    const int rc = min(rr, m - 1);
    double a[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) a[c] = c < k ? Lj[(int64_t)min(c, k - 1) * m + rc] : 0.0;
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
      if (c >= k) continue;
      double o = 0.0;
#pragma unroll
      for (int u = 0; u <= c; ++u) o = fma(a[u], readlane_d(x[c / MB][c % MB], ub + u), o);
      a[c] = o;
    }
    if (ok) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < k) Lj[(int64_t)c * m + rr] = a[c];
    }
  }
}

// ---------------------------------------------------------------------------
// solves.  y is the permuted right-hand side block, n x nrhs, ld = n.
// ---------------------------------------------------------------------------

__global__ void k_perm_gather(const int64_t* __restrict__ perm, int64_t n, const double* __restrict__ B,
                              int64_t ldb, int64_t nrhs, double* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) {
    const int64_t c = i / n, r = i % n;
    y[i] = B[c * ldb + perm[r]];
  }
}

__global__ void k_perm_scatter(const int64_t* __restrict__ perm, int64_t n, const double* __restrict__ y,
                               int64_t nrhs, double* __restrict__ B, int64_t ldb) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) {
    const int64_t c = i / n, r = i % n;
    B[c * ldb + perm[r]] = y[i];
  }
}

// forward: y_p <- D_p^{-1} y_p, one wavefront per (J, panel); lane i owns
// row i, column sweep: y_j is final, broadcast with readlane, subtracted
// from the rows below
// Forward round, one task per 64-row tile below a panel (Sec. II: the
// supernodal forward substitution).  Every task forms z_p = W_p y_p with the
// stored inverse of the panel's diagonal block (y_p is final: all panels and
// supernodes that update it were processed in earlier rounds), the first
// task stores z_p into x, and the tile's rows get y_R -= L_Rp z_p: plain
// updates for rows of the supernode's own later columns (one writer),
// atomics for ancestor rows (several supernodes of a level may share one).
// Both products split the panel's columns over the four wavefronts (16
// each) and sum the partial results in LDS; right-hand sides go four at a
// time, so L and W are read once per four.
__global__ __launch_bounds__(256) void k_fwd(DevSym S, const double* __restrict__ L, const double* __restrict__ winv,
                                             int64_t off, double* __restrict__ y, double* __restrict__ x,
                                             int64_t nrhs) {
  __shared__ double ys[4][NBMAX];
  __shared__ double zs[4][NBMAX];
  __shared__ double part[4][4][NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, r0 = t.b;
  const bool first = t.c == 1;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const double* __restrict__ W = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  const int64_t fcol = S.sfirst[J] + c0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int t0 = 16 * w, t1 = min(kp, t0 + 16);
  const int row = r0 + lane;
  const bool rowok = r0 >= 0 && row < m;
  // the thread's 16 entries of W and of the tile of L, the same for every
  // block of right-hand sides: loaded once, all at the start, from clamped
  // in-bounds addresses, the entries past kp / m replaced by zero where
  // used, so that no load waits behind a branch of its own
  double wr[16], lr[16];
  const int32_t grow = R[rowok ? row : 0];  // the row this lane updates
  {
    const int il = min(lane, kp - 1), rl = rowok ? row : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int tt = t0 + u, tc = min(tt, kp - 1);
      wr[u] = W[(int64_t)tc * kp + il];
      lr[u] = Lj[(int64_t)(c0 + tc) * m + rl];
    }
  }
  // one block of four right-hand sides; the first block is peeled off the
  // loop (no wait at a loop header for the loads above)
  auto block = [&](int64_t cb) {
    {
      const int64_t c = cb + w;  // thread (lane, w) loads entry lane of RHS cb + w
      ys[w][lane] = (lane < kp && c < nrhs) ? y[fcol + lane + c * S.n] : 0.0;
    }
    __syncthreads();
    double z[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double wv = (t0 + u < t1 && lane < kp) ? here(wr[u]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) z[q] = fma(wv, ys[q][t0 + u], z[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[w][q][lane] = z[q];
    __syncthreads();
    {
      const int q = w, i = lane;  // thread (lane, w) sums entry lane of RHS cb + w
      const double v = (part[0][q][i] + part[1][q][i]) + (part[2][q][i] + part[3][q][i]);
      zs[q][i] = v;
      if (first && i < kp && cb + q < nrhs) x[fcol + i + (cb + q) * S.n] = v;
    }
    __syncthreads();
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double lv = (t0 + u < t1 && rowok) ? here(lr[u]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = fma(lv, zs[q][t0 + u], a[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[w][q][lane] = a[q];
    __syncthreads();
    {
      const int q = w, i = lane;
      const int64_t c = cb + q;
      if (rowok && c < nrhs) {
        const double v = (part[0][q][i] + part[1][q][i]) + (part[2][q][i] + part[3][q][i]);
        double* dst = y + grow + c * S.n;
        if (r0 + i < k) *dst -= v;
        else atomicAdd(dst, -v);
      }
    }
    __syncthreads();
  };
  block(0);
  for (int64_t cb = 4; cb < nrhs; cb += 4) block(cb);
}

// Solve rounds of small supernodes: one panel of at most 16 columns with at
// most 128 rows below it (the leaf levels of a nested-dissection ordering,
// thousands of supernodes a level).  One wavefront per supernode, four per
// workgroup, no LDS and no barrier: lane i holds row (forward) or column
// (backward) i of the inverted diagonal block and rows k + i and
// k + 64 + i of L, and the solution entries pass from lane to lane by
// readlane.  Task: J, 0, k_J, 1.
constexpr int kSmallSolveCols = 16;

// the lane's rows below the diagonal block, clamped in bounds (row 0 when
// there is none: then unused), their global rows and entries of L
struct SmallRows {
  bool ok0, ok1;
  int32_t g0, g1;
  double l0[kSmallSolveCols], l1[kSmallSolveCols];
};

// (TWO = false: at most 64 rows below, the second chunk left out altogether,
// its registers too)
template <bool TWO>
__device__ __forceinline__ void small_rows(const DevSym& S, const double* __restrict__ Lj, int J, int m, int k,
                                           int lane, SmallRows& r) {
  const int nbl = m - k;
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  r.ok0 = lane < nbl;
  r.ok1 = TWO && TILE + lane < nbl;
  const int rl0 = nbl > 0 ? k + min(lane, nbl - 1) : 0;
  r.g0 = R[rl0];
#pragma unroll
  for (int u = 0; u < kSmallSolveCols; ++u) r.l0[u] = Lj[(int64_t)min(u, k - 1) * m + rl0];
  // a second chunk of rows only where the supernode has one (a branch
  // uniform over the wavefront)
  r.g1 = 0;
#pragma unroll
  for (int u = 0; u < kSmallSolveCols; ++u) r.l1[u] = 0.0;
  if (TWO && nbl > TILE) {
    const int rl1 = k + TILE + min(lane, nbl - TILE - 1);
    r.g1 = R[rl1];
#pragma unroll
    for (int u = 0; u < kSmallSolveCols; ++u) r.l1[u] = Lj[(int64_t)min(u, k - 1) * m + rl1];
  }
}

// Forward: z = W y_J, stored into x; y_R -= L_RJ z with atomics (the rows
// below are ancestors', shared with other supernodes of the level).
template <bool TWO>
__global__ __launch_bounds__(256) void k_fwd_small(DevSym S, const double* __restrict__ L,
                                                   const double* __restrict__ winv, int64_t off, int32_t ntasks,
                                                   double* __restrict__ y, double* __restrict__ x, int64_t nrhs) {
  const int lane = threadIdx.x & 63;
  const int ti = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ti >= ntasks) return;
  const int J = S.tasks[off + ti].J;
  const int m = S.sm[J], k = S.sk[J];
  const double* __restrict__ Lj = L + S.loff[J];
  const double* __restrict__ W = winv + S.wbase[J];
  const int64_t fcol = S.sfirst[J];
  const bool own = lane < k;
  const int il = min(lane, k - 1);  // the lane's row of W (clamped)
  double wr[kSmallSolveCols];
#pragma unroll
  for (int u = 0; u < kSmallSolveCols; ++u) wr[u] = W[min(u, k - 1) * k + il];
  SmallRows rw;
  small_rows<TWO>(S, Lj, J, m, k, lane, rw);
  // right-hand sides four at a time: the group's entries of y_J are all
  // loaded before the first product (one memory round trip per group)
  for (int64_t cb = 0; cb < nrhs; cb += 4) {
    double yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] = (own && cb + q < nrhs) ? y[fcol + lane + (cb + q) * S.n] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t c = cb + q;
      if (c >= nrhs) break;
      double z = 0.0;
#pragma unroll
      for (int u = 0; u < kSmallSolveCols; ++u) z = fma(u < k ? wr[u] : 0.0, readlane_d(yv[q], u), z);
      z = own ? z : 0.0;
      if (own) x[fcol + lane + c * S.n] = z;
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int u = 0; u < kSmallSolveCols; ++u) {
        const double zu = readlane_d(z, u);
        a0 = fma(u < k ? rw.l0[u] : 0.0, zu, a0);
        a1 = fma(u < k ? rw.l1[u] : 0.0, zu, a1);
      }
      if (rw.ok0) atomicAdd(y + rw.g0 + c * S.n, -a0);
      if (rw.ok1) atomicAdd(y + rw.g1 + c * S.n, -a1);
    }
  }
}

// One step of the transposing butterfly below: a lane keeps half of its h
// partial column sums, hands the other half to the partner lane (lane ^
// msk) and adds the partner's half of its own.
template <int H, int MSK>
__device__ __forceinline__ void col_sum_step(double (&v)[kSmallSolveCols], int lane) {
  const bool hi = (lane & MSK) != 0;
#pragma unroll
  for (int u = 0; u < H; ++u) {
    const double send = hi ? v[u] : v[u + H];
    const double keep = hi ? v[u + H] : v[u];
    v[u] = keep + __shfl_xor(send, MSK);
  }
}

// Column sums over the wavefront of v[u] (u = column): returns, in lane l,
// the total of column 8 b5 + 4 b4 + 2 b3 + b2 (b_i: bit i of l).  After the
// four halving steps a lane holds that column summed over the 16 lanes that
// differ from it in bits 5..2; two exchanges add the other three groups.
__device__ __forceinline__ double col_sums16(double (&v)[kSmallSolveCols], int lane) {
  col_sum_step<8, 32>(v, lane);
  col_sum_step<4, 16>(v, lane);
  col_sum_step<2, 8>(v, lane);
  col_sum_step<1, 4>(v, lane);
  double s = v[0];
  s += __shfl_xor(s, 2);
  s += __shfl_xor(s, 1);
  return s;
}

// the lane that holds column u after col_sums16
__device__ __forceinline__ constexpr int col_sum_lane(int u) {
  return ((u >> 3) & 1) * 32 + ((u >> 2) & 1) * 16 + ((u >> 1) & 1) * 8 + (u & 1) * 4;
}

// Backward: x_J = W^T (x_J - L_RJ^T x_R) (x_R final: ancestors are done in
// earlier rounds).
template <bool TWO>
__global__ __launch_bounds__(256) void k_bwd_small(DevSym S, const double* __restrict__ L,
                                                   const double* __restrict__ winv, int64_t off, int32_t ntasks,
                                                   double* __restrict__ x, int64_t nrhs) {
  const int lane = threadIdx.x & 63;
  const int ti = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ti >= ntasks) return;
  const int J = S.tasks[off + ti].J;
  const int m = S.sm[J], k = S.sk[J];
  const double* __restrict__ Lj = L + S.loff[J];
  const double* __restrict__ W = winv + S.wbase[J];
  const int64_t fcol = S.sfirst[J];
  const bool own = lane < k;
  const int il = min(lane, k - 1);
  // wt[u] = W_{u, lane} (column `lane` of W)
  double wt[kSmallSolveCols];
#pragma unroll
  for (int u = 0; u < kSmallSolveCols; ++u) wt[u] = W[il * k + min(u, k - 1)];
  SmallRows rw;
  small_rows<TWO>(S, Lj, J, m, k, lane, rw);
  for (int64_t c = 0; c < nrhs; ++c) {
    const double xr0 = rw.ok0 ? x[rw.g0 + c * S.n] : 0.0;
    const double xr1 = rw.ok1 ? x[rw.g1 + c * S.n] : 0.0;
    const double xf = own ? x[fcol + lane + c * S.n] : 0.0;
    double v[kSmallSolveCols];
#pragma unroll
    for (int u = 0; u < kSmallSolveCols; ++u)
      v[u] = u < k ? fma(rw.ok0 ? rw.l0[u] : 0.0, xr0, (rw.ok1 ? rw.l1[u] : 0.0) * xr1) : 0.0;
    const double s = col_sums16(v, lane);
    double r = 0.0;
#pragma unroll
    for (int u = 0; u < kSmallSolveCols; ++u)
      r = fma(u < k ? wt[u] : 0.0, readlane_d(xf, u) - readlane_d(s, col_sum_lane(u)), r);
    if (own) x[fcol + lane + c * S.n] = r;
  }
}

// Forward round with two-panel tasks (c bit 1; single-panel tasks of
// supernodes whose last panel is p run as in k_fwd): z_p = W_p y_p, the
// right-hand side of panel p + 1 less the coupling block's share,
// t = y_{p+1} - L_{p+1,p} z_p, then z_{p+1} = W_{p+1} t; the first task
// stores both, and the tile below panel p + 1 gets
// y_R -= L_Rp z_p + L_R,p+1 z_{p+1}.  One launch instead of two for the
// panel pair; the same thread layout as k_fwd (wavefront w: columns 16w..,
// lane: row), every load issued at the start.
__global__ __launch_bounds__(256) void k_fwd2(DevSym S, const double* __restrict__ L, const double* __restrict__ winv,
                                              int64_t off, double* __restrict__ y, double* __restrict__ x,
                                              int64_t nrhs) {
  __shared__ double ys[4][NBMAX], ys1[4][NBMAX];
  __shared__ double zs[4][NBMAX], zs1[4][NBMAX];
  __shared__ double part[4][4][NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, r0 = t.b;
  const bool first = (t.c & 1) != 0, dbl = (t.c & 2) != 0;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const int c1 = c0 + kp, kp1 = dbl ? min(S.nb, k - c1) : 1;  // (1: a valid clamp when single)
  const double* __restrict__ Lj = L + S.loff[J];
  const double* __restrict__ W = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;
  const double* __restrict__ W1 = dbl ? W + (int64_t)S.nb * S.nb : W;
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  const int64_t fcol = S.sfirst[J] + c0, fcol1 = fcol + kp;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int t0 = 16 * w, t1 = min(kp, t0 + 16), t1b = dbl ? min(kp1, t0 + 16) : 0;
  const int row = r0 + lane;
  const bool rowok = r0 >= 0 && row < m;
  const int32_t grow = R[rowok ? row : 0];
  double wr[16], lr[16], wr1[16], lc[16], lr1[16];
  {
    const int il = min(lane, kp - 1), il1 = min(lane, kp1 - 1), rl = rowok ? row : 0;
    const int rc = min(c1 + lane, m - 1);  // (a row of panel p + 1 when double)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int tt = t0 + u, tc = min(tt, kp - 1), tc1 = min(tt, kp1 - 1);
      wr[u] = W[(int64_t)tc * kp + il];
      lr[u] = Lj[(int64_t)(c0 + tc) * m + rl];
      wr1[u] = W1[(int64_t)tc1 * kp1 + il1];
      lc[u] = Lj[(int64_t)(c0 + tc) * m + rc];
      lr1[u] = Lj[(int64_t)(dbl ? c1 + tc1 : c0 + tc) * m + rl];
    }
  }
  // sum over the four wavefronts of v (thread (lane, w): RHS q, entry lane)
  auto reduce = [&](const double (&v)[4], double (*out)[NBMAX]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) part[w][q][lane] = v[q];
    __syncthreads();
    out[w][lane] = (part[0][w][lane] + part[1][w][lane]) + (part[2][w][lane] + part[3][w][lane]);
    __syncthreads();
  };
  auto block = [&](int64_t cb) {
    {
      const int64_t c = cb + w;  // thread (lane, w) loads entry lane of RHS cb + w
      ys[w][lane] = (lane < kp && c < nrhs) ? y[fcol + lane + c * S.n] : 0.0;
      ys1[w][lane] = (dbl && lane < kp1 && c < nrhs) ? y[fcol1 + lane + c * S.n] : 0.0;
    }
    __syncthreads();
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double a = (t0 + u < t1 && lane < kp) ? here(wr[u]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = fma(a, ys[q][t0 + u], v[q]);
    }
    reduce(v, zs);  // z_p
    if (first && lane < kp && cb + w < nrhs) x[fcol + lane + (cb + w) * S.n] = zs[w][lane];
    if (dbl) {
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double a = (t0 + u < t1 && lane < kp1) ? here(lc[u]) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = fma(a, zs[q][t0 + u], v[q]);
      }
      reduce(v, part[0]);  // (the coupling block's share, in a free slot)
      ys1[w][lane] -= part[0][w][lane];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double a = (t0 + u < t1b && lane < kp1) ? here(wr1[u]) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = fma(a, ys1[q][t0 + u], v[q]);
      }
      reduce(v, zs1);  // z_{p+1}
      if (first && lane < kp1 && cb + w < nrhs) x[fcol1 + lane + (cb + w) * S.n] = zs1[w][lane];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const double a = (t0 + u < t1 && rowok) ? here(lr[u]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = fma(a, zs[q][t0 + u], v[q]);
    }
    if (dbl) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const double a = (t0 + u < t1b && rowok) ? here(lr1[u]) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = fma(a, zs1[q][t0 + u], v[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[w][q][lane] = v[q];
    __syncthreads();
    {
      const int q = w, i = lane;
      const int64_t c = cb + q;
      if (rowok && c < nrhs) {
        const double sv = (part[0][q][i] + part[1][q][i]) + (part[2][q][i] + part[3][q][i]);
        double* dst = y + grow + c * S.n;
        if (r0 + i < k) *dst -= sv;
        else atomicAdd(dst, -sv);
      }
    }
    __syncthreads();
  };
  block(0);
  for (int64_t cb = 4; cb < nrhs; cb += 4) block(cb);
}

// The panel's inverted diagonal block (kp x kp, column-major) into LDS,
// Ws[c][r] = W_rc, zero past kp; coalesced.
__device__ __forceinline__ void stage_w(const double* __restrict__ W, int kp, double (*Ws)[NBMAX + 1], int tid,
                                        int nthr) {
  for (int idx = tid; idx < NBMAX * NBMAX; idx += nthr) {
    const int c = idx >> 6, r = idx & 63;
    Ws[c][r] = (c < kp && r < kp) ? W[c * kp + r] : 0.0;
  }
}

// (W^T v)_i = sum_tt W_tt,i v_tt = sum_tt Ws[i][tt] vs[tt] (W lower
// triangular, zero padded: the full sum is exact)
__device__ __forceinline__ double apply_wt(double (*Ws)[NBMAX + 1], const double* __restrict__ vs, int i) {
  double z = 0.0;
#pragma unroll 16
  for (int tt = 0; tt < NBMAX; ++tt) z = fma(Ws[i][tt], vs[tt], z);
  return z;
}

// Backward round (Sec. II: the supernodal back substitution).  c = -1: the
// task gathers L_Rp^T x_R over all rows below the panel (x_R is final:
// later panels and ancestors were done in earlier rounds), then forms
// x_p = W_p^T (x_p - L_Rp^T x_R).  c = 0: the task adds the share of one
// 64-row tile into acc_p (a round ahead of the panel).  c = 1 + n: the
// task gathers the n rows from rb (the next panel's, finished in the round
// before), subtracts acc_p, leaves acc_p at zero for the next solve and
// finishes the panel.  Each 64-row chunk of L is staged in LDS (coalesced)
// once per four right-hand sides; thread (lane, w) sums column lane over
// rows 16w..16w+15.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_bwd(DevSym S, const double* __restrict__ L, const double* __restrict__ winv,
                                             int64_t off, double* __restrict__ x, double* __restrict__ acc,
                                             int64_t nrhs) {
  __shared__ double Ls[TILE][NBMAX + 1];
  __shared__ double xs[4][TILE];
  __shared__ double red[4][4][NBMAX];
  __shared__ double vs[4][NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, rb = t.b;
  const bool fin = t.c != 0, useacc = t.c > 0;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  const int64_t fcol = S.sfirst[J] + c0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int re = t.c < 0 ? m : (t.c == 0 ? min(m, rb + TILE) : rb + t.c - 1);
  // a finishing task loads the panel's inverse block at the start (thread
  // tid holds entries u * 256 + tid, column-major, zero past kp), beside the
  // gather's loads rather than after them
  double wv[NBMAX * NBMAX / 256];
  if (fin) {
    const double* __restrict__ W = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;
#pragma unroll
    for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
      const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
      wv[u] = W[min(c, kp - 1) * kp + min(r, kp - 1)];  // (replaced past kp when staged)
    }
  }
  // one block of four right-hand sides, and in it one 64-row chunk; the
  // first block and its first chunk are peeled off the loops (no wait at a
  // loop header for the loads issued before)
  auto block = [&](int64_t cb) {
    // this block's entries of x_p and acc_p for thread (lane, w), issued
    // before the gather
    const int64_t cq = cb + w;
    const bool okq = lane < kp && cq < nrhs;
    const int64_t eq = fcol + (okq ? lane + cq * S.n : 0);
    const double xq = fin ? x[eq] : 0.0;
    const double aq = useacc ? acc[eq] : 0.0;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    auto chunk = [&](int r0) {
      const int nr = min(TILE, re - r0);
      const int32_t gr = R[r0 + min(lane, nr - 1)];  // row lane of the chunk (clamped)
      double lv[TILE * NBMAX / 256];
#pragma unroll
      for (int u = 0; u < TILE * NBMAX / 256; ++u) {
        const int idx = u * 256 + tid, r = idx & (TILE - 1), tt = idx / TILE;
        lv[u] = Lj[(int64_t)(c0 + min(tt, kp - 1)) * m + r0 + min(r, nr - 1)];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < TILE * NBMAX / 256; ++u) {
        const int idx = u * 256 + tid, r = idx & (TILE - 1), tt = idx / TILE;
        Ls[r][tt] = (r < nr && tt < kp) ? here(lv[u]) : 0.0;
      }
      {
        const int64_t c = cb + w;  // thread (lane, w) loads row lane for RHS cb + w
        xs[w][lane] = (lane < nr && c < nrhs) ? x[gr + c * S.n] : 0.0;
      }
      __syncthreads();
      if (lane < kp)
        for (int r = 16 * w; r < 16 * w + 16; ++r) {
          const double lv = Ls[r][lane];
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = fma(lv, xs[q][r], a[q]);
        }
    };
    if (rb < re) chunk(rb);
    for (int r0 = rb + TILE; r0 < re; r0 += TILE) chunk(r0);
#pragma unroll
    for (int q = 0; q < 4; ++q) red[w][q][lane] = a[q];
    __syncthreads();
    {
      const int q = w, i = lane;  // thread (lane, w): entry lane of RHS cb + w
      const double v = (red[0][q][i] + red[1][q][i]) + (red[2][q][i] + red[3][q][i]);
      if (useacc && okq) acc[eq] = 0.0;
      if (fin) vs[q][i] = okq ? xq - (v + aq) : 0.0;
      else if (okq) atomicAdd(acc + eq, v);
    }
    __syncthreads();
    if (fin) {
#pragma unroll
      for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
        const int idx = u * 256 + tid, c = idx >> 6, r = idx & 63;
        Ls[c][r] = (c < kp && r < kp) ? here(wv[u]) : 0.0;
      }
      __syncthreads();
      if (okq) x[eq] = apply_wt(Ls, vs[w], lane);
    }
  };
  block(0);
  for (int64_t cb = 4; cb < nrhs; cb += 4) block(cb);
}

// ---------------------------------------------------------------------------
// logdet = 2 sum_j log L_jj: per-block tree sums, then one block.
// ---------------------------------------------------------------------------

__device__ inline double block_sum_256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(256) void k_logdet_partial(DevSym S, const double* __restrict__ L,
                                                        double* __restrict__ partial) {
  __shared__ double sh[256];
  const int64_t j = blockIdx.x * (int64_t)256 + threadIdx.x;
  double v = 0.0;
  if (j < S.n) {
    const int J = S.snode_of[j];
    const int64_t d = j - S.sfirst[J];
    v = log(L[S.loff[J] + d * S.sm[J] + d]);
  }
  const double s = block_sum_256(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_logdet_final(const double* __restrict__ partial, int32_t np,
                                                      double* __restrict__ out) {
  __shared__ double sh[256];
  // contiguous chunks per thread keep the summation tree-shaped
  const int per = (np + 255) / 256;
  const int b = threadIdx.x * per;
  double v = 0.0;
  for (int i = b; i < min(np, b + per); ++i) v += partial[i];
  const double s = block_sum_256(v, sh);
  if (threadIdx.x == 0) *out = 2.0 * s;
}

// ---------------------------------------------------------------------------
// reverse mode: selected inversion Z = C^{-1} on the supernodal pattern of L
// (C = P A P^T), stored in the layout of L.  From Z L = L^{-T} (upper
// triangular) follow, for a panel p of supernode J (columns c0..c0+kp) with
// the rows B of J below it:
//   Z_Bp = -Z_BB L_Bp L_pp^{-1},      Z_pp = (W^T - Z_Bp^T L_Bp) W,
// with W = L_pp^{-1}.  Panels are visited root to leaves and, inside a
// supernode, last panel first, so Z_BB (later columns of J, then ancestors
// reached through the relative indices) is final when needed.  Per panel:
//   k_si_y   Y = Z_BB L_Bp, 64-row tiles, Z_BB gathered (symmetric), split
//            over segments of B and summed into Y;
//   k_si_zb  Z_Bp = -Y W per tile, and T += Z_Bp^T L_Bp (atomic);
//   k_si_zd  Z_pp = (W^T - T) W, lower part.
// W is the inverted diagonal block the factorization stored.  Y and T are
// zero on entry to a round: k_si_zb clears the Y rows it read, k_si_zd the
// T it read.  Task fields: J, panel, first local row of the tile, slot in
// the round.
// ---------------------------------------------------------------------------

// offset in Z (layout of L) of the symmetric entry at local rows (a, b) of
// J, both at or below J's first column
// Where Z(lo, hi) (lo <= hi, local rows of J) lives: the column of row lo
// is either J's own (lo < k) or an ancestor's, whose storage column starts
// at colbase; the entry of row hi in it is at colbase + hi (lo < k) or
// colbase + tpos[tb + hi - k] (the relative index of hi in the ancestor).
struct ZCol {
  int64_t colbase;
  int64_t tb;  // relptr[pair] - pa0[pair], or -1 for J's own columns
};

__device__ __forceinline__ ZCol zcol(const DevSym& S, int J, int k, int m, int64_t ob, int lo) {
  if (lo < k) return ZCol{S.loff[J] + (int64_t)lo * m, -1};
  const int pair = S.opair[ob + lo - k];
  return ZCol{S.ocbase[ob + lo - k], S.relptr[pair] - S.pa0[pair]};
}

__device__ __forceinline__ int64_t zat(const DevSym& S, ZCol c, int k, int hi) {
  return c.colbase + (c.tb < 0 ? (int64_t)hi : (int64_t)S.tpos[c.tb + hi - k]);
}

// Y[a][t] = sum_{b in B} Z(a, b) L[b][c0 + t] for a in [a0, a0 + 64), each
// task over one segment of seglen (<= kSiSeg) rows b of B (Y zeroed
// beforehand).  The
// column data of the tile's rows a is fetched once; that of each K chunk's
// 16 rows b once per chunk into LDS, so an entry of Z costs one relative
// index load and the entry itself.
__global__ __launch_bounds__(256) void k_si_y(DevSym S, const double* __restrict__ L, const double* __restrict__ Z,
                                              int64_t off, const int64_t* __restrict__ yoff,
                                              double* __restrict__ ybuf, int seglen) {
  __shared__ double As[KC * ALD];
  __shared__ double Bs[KC * ALD];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a & 0xFFFF, seg = t.a >> 16, a0 = t.b, slot = t.c;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const int rb = c0 + kp;
  const int bs = rb + seg * seglen, be = min(m, bs + seglen);  // this task's rows of B
  const double* __restrict__ Lj = L + S.loff[J];
  const int64_t ob = S.obase[J];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const int sr = tid & 63, sc = tid >> 6;
  const int a = a0 + sr;
  // Z is stored by columns (lower part): Z(a, b) with a >= b is read down
  // column b (consecutive a contiguous), with a < b down column a
  // (consecutive b contiguous).  Chunks entirely above the tile's diagonal
  // therefore use a transposed thread mapping (16 lanes along b).  The
  // column data of the tile's rows and of all rows of the segment are
  // fetched once; the next chunk's entries are loaded into registers while
  // the current one is multiplied.
  __shared__ ZCol cola[TILE];
  __shared__ ZCol colseg[kSiSeg];
  if (tid < TILE) cola[tid] = a0 + tid < m ? zcol(S, J, k, m, ob, a0 + tid) : ZCol{0, -1};
  for (int i = tid; i < kSiSeg; i += 256) colseg[i] = bs + i < be ? zcol(S, J, k, m, ob, bs + i) : ZCol{0, -1};
  __syncthreads();
  const ZCol ca = a < m ? cola[sr] : ZCol{0, -1};
  // The loads of a chunk are issued together: the positions of the
  // ancestor-column entries first, then the entries of Z and of L, all from
  // clamped in-bounds indices; entries past the tile / segment are replaced
  // by zero when staged (masks ma, mb).
  double ra[4], rbv[4];
  bool ma[4], mb[4];
  auto fetch = [&](int b0) {
    int64_t zb[4], ti[4];
    int hv[4];
    bool rl[4];
    if (b0 >= a0 + TILE - 1) {  // every b of the chunk >= every a of the tile
      const int bi = tid & (KC - 1), b = b0 + bi;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ai = (tid >> 4) + 16 * q;
        const ZCol c = cola[ai];
        ma[q] = a0 + ai < m && b < be;
        zb[q] = c.colbase;
        rl[q] = c.tb >= 0;
        hv[q] = b;
        ti[q] = c.tb + b - k;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = b0 + sc + 4 * q;
        const ZCol c = a >= b ? colseg[min(b - bs, kSiSeg - 1)] : ca;
        const int hi = a >= b ? a : b;
        ma[q] = a < m && b < be;
        zb[q] = c.colbase;
        rl[q] = c.tb >= 0;
        hv[q] = hi;
        ti[q] = c.tb + hi - k;
      }
    }
    int tp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) tp[q] = S.tpos[(ma[q] && rl[q]) ? ti[q] : 0];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + sc + 4 * q;
      mb[q] = b < be && sr < kp;
      rbv[q] = Lj[(int64_t)(c0 + min(sr, kp - 1)) * m + min(b, be - 1)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = Z[ma[q] ? zb[q] + (rl[q] ? (int64_t)tp[q] : (int64_t)hv[q]) : 0];
  };
  fetch(bs);
  for (int b0 = bs; b0 < be; b0 += KC) {
    if (b0 >= a0 + TILE - 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) As[(tid & (KC - 1)) * ALD + (tid >> 4) + 16 * q] = ma[q] ? here(ra[q]) : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) As[(sc + 4 * q) * ALD + sr] = ma[q] ? here(ra[q]) : 0.0;  // As[kb][a - a0]
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[(sc + 4 * q) * ALD + sr] = mb[q] ? here(rbv[q]) : 0.0;  // Bs[kb][t]
    __syncthreads();
    if (b0 + KC < be) fetch(b0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = (ks + lk) * ALD;
      const double x0 = As[kr + wr + li], x1 = As[kr + wr + 16 + li];
      const double y0 = Bs[kr + wc + li], y1 = Bs[kr + wc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* __restrict__ Y = ybuf + yoff[slot];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int tc = wc + 16 * bj + li;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ar = a0 + wr + 16 * bi + 4 * v + lk;
        if (ar < m && tc < kp) atomicAdd(Y + (int64_t)(ar - rb) * NBMAX + tc, acc[bi][bj][v]);
      }
  }
}

// Z_Bp = -Y W on rows [a0, a0 + 64), and T += Z_Bp^T L_Bp
__global__ __launch_bounds__(256) void k_si_zb(DevSym S, const double* __restrict__ L, const double* __restrict__ winv,
                                               double* __restrict__ Z, int64_t off, const int64_t* __restrict__ yoff,
                                               double* __restrict__ ybuf, double* __restrict__ tbuf) {
  __shared__ __attribute__((aligned(16))) double As[NBMAX * DLD];
  __shared__ __attribute__((aligned(16))) double Wc[NBMAX * DLD];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, a0 = t.b, slot = t.c;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const int rb = c0 + kp;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double* __restrict__ Y = ybuf + yoff[slot];
  const double* __restrict__ W = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;  // kp x kp, column-major
  const double* __restrict__ Lp = L + S.loff[J] + (int64_t)c0 * m;
  double* __restrict__ Zp = Z + S.loff[J] + (int64_t)c0 * m;
  // every load at the start, from clamped in-bounds addresses (entries
  // past the block replaced by zero when staged): the Y block (row-major),
  // W, and the tile of L_Bp for T
  double yv[NBMAX * NBMAX / 256], wv[NBMAX * NBMAX / 256], lv[NBMAX * NBMAX / 256];
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx >> 6, c = idx & 63;
    yv[u] = Y[(int64_t)(min(a0 + r, m - 1) - rb) * NBMAX + c];
    wv[u] = W[min(c, kp - 1) * kp + min(r, kp - 1)];
    lv[u] = Lp[(int64_t)min(r, kp - 1) * m + min(a0 + c, m - 1)];  // (row a0 + c, column r)
  }
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx >> 6, c = idx & 63;
    const bool iny = a0 + r < m;
    As[c * DLD + r] = (iny && c < kp) ? here(yv[u]) : 0.0;
    if (iny) Y[(int64_t)(a0 + r - rb) * NBMAX + c] = 0.0;  // leave Y cleared for the next round
    // V = W^T column-major: Wc[c * DLD + i] = V_ic = W_ci, i.e. Wc[r * DLD + c] = W_rc
    Wc[r * DLD + c] = (r < kp && c < kp) ? here(wv[u]) : 0.0;
  }
  __syncthreads();
  // Z_Bp = -(Y V^T) = -(Y W); wavefront w: columns 16w.., rows 16 rb2 + 4v + lk
  const bool act = MB * w < kp;
  const int li = lane & 15, lk = lane >> 4, cz = MB * w + li;
  d4 zacc[4];
  if (act) {
    tile_mfma_acc(As, Wc, kp, lane, w, zacc);
    if (cz < kp) {
#pragma unroll
      for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = 16 * rb2 + 4 * v + lk;
          if (a0 + rr < m) Zp[(int64_t)cz * m + a0 + rr] = -zacc[rb2][v];
        }
    }
  }
  __syncthreads();
  // T partial: the Z tile (column-major, zero past m / kp) from the
  // accumulators into As, the L_Bp tile into Wc
#pragma unroll
  for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = 16 * rb2 + 4 * v + lk;
      As[cz * DLD + rr] = (act && cz < kp && a0 + rr < m) ? -zacc[rb2][v] : 0.0;
    }
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx >> 6, c = idx & 63;
    Wc[r * DLD + c] = (a0 + c < m && r < kp) ? here(lv[u]) : 0.0;
  }
  __syncthreads();
  // T[s][c] = sum_r Z[r][s] L[r][c]: A operand A[s][r] = Z[r][s] = As[s * DLD + r],
  // B operand B[r][c] = L[r][c] = Wc[c * DLD + r]; wavefront w owns columns 16w..
  if (MB * w < kp) {
    d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < NBMAX; r0 += 4) {
      const double bv = Wc[(MB * w + li) * DLD + r0 + lk];
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const double av = As[(16 * sb + li) * DLD + r0 + lk];
        acc[sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[sb], 0, 0, 0);
      }
    }
    double* Tt = tbuf + (int64_t)slot * NBMAX * NBMAX;
    const int c = MB * w + li;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = 16 * sb + 4 * v + lk;
        if (s < kp && c < kp) atomicAdd(Tt + s * NBMAX + c, acc[sb][v]);
      }
  }
}

// Z_pp = (W^T - T) W, lower part
__global__ __launch_bounds__(256) void k_si_zd(DevSym S, const double* __restrict__ winv, double* __restrict__ Z,
                                               int64_t off, double* __restrict__ tbuf) {
  __shared__ __attribute__((aligned(16))) double As[NBMAX * DLD];
  __shared__ __attribute__((aligned(16))) double Wc[NBMAX * DLD];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, slot = t.c;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* __restrict__ W = winv + S.wbase[J] + (int64_t)p * S.nb * S.nb;  // kp x kp, column-major
  double* __restrict__ T = tbuf + (int64_t)slot * NBMAX * NBMAX;
  // every load at the start (clamped, entries past kp replaced by zero)
  double w1[NBMAX * NBMAX / 256], w2[NBMAX * NBMAX / 256], tv[NBMAX * NBMAX / 256];
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx >> 6, c = idx & 63;
    w1[u] = W[min(r, kp - 1) * kp + min(c, kp - 1)];
    w2[u] = W[min(c, kp - 1) * kp + min(r, kp - 1)];
    tv[u] = T[idx];
  }
#pragma unroll
  for (int u = 0; u < NBMAX * NBMAX / 256; ++u) {
    const int idx = u * 256 + tid, r = idx >> 6, c = idx & 63;
    const bool in = r < kp && c < kp;
    // M = W^T - T column-major: As[c * DLD + r] = W[c][r] - T[r][c]
    As[c * DLD + r] = (in ? here(w1[u]) : 0.0) - here(tv[u]);
    T[idx] = 0.0;  // leave T cleared for the next round
    Wc[r * DLD + c] = in ? here(w2[u]) : 0.0;  // V = W^T column-major: Wc[r * DLD + c] = W_rc
  }
  __syncthreads();
  double* __restrict__ Zp = Z + S.loff[J] + (int64_t)c0 * m;
  tile_mfma(As, Wc, kp, lane, w, Zp, m, c0, c0 + kp, true, 1.0);
}

// Abar for every stored entry p = (i, j) of A (original ordering):
//   Abar_p = g w_p Z(i, j) - sum_c (lam_ic x_jc + [i != j] lam_jc x_ic),
// w_p = 2 off the diagonal (the entry stands for a_ij and a_ji), 1 on it.
__global__ void k_abar(const DevSym S, const double* __restrict__ Z, double g, const double* __restrict__ X,
                       const double* __restrict__ lam, int64_t ld, int64_t nrhs, double* __restrict__ Abar) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; q < S.nnzA; q += stride) {
    const int i = S.e_row[q], j = S.e_col[q];
    double s = 0.0;
    if (Z) s = g * (i != j ? 2.0 : 1.0) * Z[S.amap[q]];
    if (lam) {
      for (int64_t c = 0; c < nrhs; ++c) {
        s -= lam[i + c * ld] * X[j + c * ld];
        if (i != j) s -= lam[j + c * ld] * X[i + c * ld];
      }
    }
    Abar[q] = s;
  }
}

// ---------------------------------------------------------------------------
// iterative refinement against the fp64 matrix (original ordering).  A is
// applied from its stored lower triangle through a full-symmetric CSR whose
// entries index the value array (gather, no atomics).  Norm reductions keep
// non-negative doubles as their bit patterns (monotone as unsigned).
// stats[3c + 0] = max_i |r_i|, [3c + 1] = max_i |x_i|, [3c + 2] = max_i |b_i|.
// ---------------------------------------------------------------------------

__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int64_t count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

// Rows of A (full-symmetric CSR) are read by groups of 16 lanes, 16 rows
// at a time per workgroup (coalesced runs of each row's entries); maxima are
// reduced in the workgroup and added with one atomic per workgroup and
// statistic.
constexpr int kRowLanes = 16;

// Maxima of NV values over the workgroup (wavefront exchanges, one LDS
// step); thread t < NV returns the maximum of value t, the others 0.
template <int NV>
__device__ __forceinline__ double block_max_multi(const double (&v)[NV], double (*sh)[NV]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double m = v[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) sh[w][j] = m;
  }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < NV) {
    const int j = threadIdx.x;
    r = fmax(fmax(sh[0][j], sh[1][j]), fmax(sh[2][j], sh[3][j]));
  }
  __syncthreads();
  return r;
}

// ||A||_inf = max_i sum_j |a_ij|.  Each 16-lane group takes rows
// blockIdx.x * 16 + group, stepping by the grid: the workgroup's maximum
// then costs one atomic (a grid of at most kStatBlocks workgroups keeps
// the atomics on the one word few).
constexpr int kStatBlocks = 1024;
__global__ __launch_bounds__(256) void k_anorm(const int64_t* __restrict__ rp, const int64_t* __restrict__ vidx,
                                               const double* __restrict__ vals, int64_t n,
                                               unsigned long long* __restrict__ out) {
  __shared__ double sh[4][1];
  const int g = threadIdx.x % kRowLanes;
  double m[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)(256 / kRowLanes) + threadIdx.x / kRowLanes; i < n;
       i += (int64_t)gridDim.x * (256 / kRowLanes)) {
    double s = 0.0;
    for (int64_t q = rp[i] + g; q < rp[i + 1]; q += kRowLanes) s += fabs(vals[vidx[q]]);
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kRowLanes);
    m[0] = fmax(m[0], s);
  }
  const double r = block_max_multi<1>(m, sh);
  if (threadIdx.x == 0) atomic_max_nonneg(out, r);
}

// R = B - A X for nrhs columns (B == NULL: R = -A X), with the normwise
// statistics max|R|, max|X|, max|B| per column; each entry of A is read
// once per four columns.  Rows by 16-lane groups, stepping by the grid as
// in k_anorm; per block of four columns the workgroup's twelve maxima go
// out with one atomic each.
__global__ __launch_bounds__(256) void k_residual(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const int64_t* __restrict__ vidx, const double* __restrict__ vals,
                                                  int64_t n, const double* __restrict__ B, int64_t ldb,
                                                  const double* __restrict__ X, int64_t ldx, int64_t nrhs,
                                                  double* __restrict__ R, unsigned long long* __restrict__ stats) {
  __shared__ double sh[4][12];
  const int g = threadIdx.x % kRowLanes;
  for (int64_t cb = 0; cb < nrhs; cb += 4) {
    double mm[12];  // max |r|, |x|, |b| of columns cb + u at 3u, 3u + 1, 3u + 2
#pragma unroll
    for (int j = 0; j < 12; ++j) mm[j] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)(256 / kRowLanes) + threadIdx.x / kRowLanes; i < n;
         i += (int64_t)gridDim.x * (256 / kRowLanes)) {
      const int64_t q0 = rp[i], q1 = rp[i + 1];
      double s[4] = {0.0, 0.0, 0.0, 0.0};
      for (int64_t q = q0 + g; q < q1; q += kRowLanes) {
        const double a = vals[vidx[q]];
        const int64_t j = col[q];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (cb + u < nrhs) s[u] = fma(-a, X[(cb + u) * ldx + j], s[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int o = kRowLanes / 2; o > 0; o >>= 1) s[u] += __shfl_xor(s[u], o, kRowLanes);
        const int64_t c = cb + u;
        if (c < nrhs) {
          const double b = B ? B[i + c * ldb] : 0.0;
          const double r = b + s[u];
          if (g == 0) R[i + c * n] = r;
          mm[3 * u] = fmax(mm[3 * u], fabs(r));
          mm[3 * u + 1] = fmax(mm[3 * u + 1], fabs(X[c * ldx + i]));
          mm[3 * u + 2] = fmax(mm[3 * u + 2], fabs(b));
        }
      }
    }
    const double r = block_max_multi<12>(mm, sh);
    if (threadIdx.x < 12 && cb + threadIdx.x / 3 < nrhs) atomic_max_nonneg(stats + 3 * cb + threadIdx.x, r);
  }
}

// Column dot products of two n x nrhs blocks (leading dimension n):
// out[c] += sum_i a[i, c] b[i, c] (out zeroed beforehand); blockIdx.y is the
// column, each workgroup one strided share of it.
__global__ __launch_bounds__(256) void k_dot_cols(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* __restrict__ out) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.y;
  double v = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    v = fma(a[i + c * n], b[i + c * n], v);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out + c, sh[0]);
}

// Y[:, c] += alpha[c] D[:, c] (Y with leading dimension ldy, D with n)
__global__ void k_axpy_cols(double* __restrict__ Y, int64_t ldy, const double* __restrict__ D, int64_t n,
                            int64_t nrhs, const double* __restrict__ alpha) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) {
    const int64_t c = i / n, r = i % n;
    Y[c * ldy + r] = fma(alpha[c], D[i], Y[c * ldy + r]);
  }
}

// P[:, c] = Z[:, c] + beta[c] P[:, c] (leading dimension n)
__global__ void k_xpby_cols(double* __restrict__ P, const double* __restrict__ Z, int64_t n, int64_t nrhs,
                            const double* __restrict__ beta) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) P[i] = fma(beta[i / n], P[i], Z[i]);
}

// X += D (n x nrhs, D with leading dimension n)
__global__ void k_axpy(double* __restrict__ X, int64_t ldx, const double* __restrict__ D, int64_t n, int64_t nrhs) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) {
    const int64_t c = i / n, r = i % n;
    X[c * ldx + r] += D[i];
  }
}

// Y (leading dimension ldy) <- B (leading dimension ldb)
__global__ void k_copy_cols(double* __restrict__ Y, int64_t ldy, const double* __restrict__ B, int64_t ldb,
                            int64_t n, int64_t nrhs) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n * nrhs; i += stride) {
    const int64_t c = i / n, r = i % n;
    Y[c * ldy + r] = B[c * ldb + r];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned grid_for(int64_t count, int64_t per = 256, int64_t cap = 16384) {
  int64_t g = (count + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_fill<<<grid_for(count), 256, 0, st>>>(p, count, v);
  return hipGetLastError();
}

hipError_t launch_status_init(unsigned long long* status, hipStream_t st) {
  k_status_init<<<1, 64, 0, st>>>(status);
  return hipGetLastError();
}

hipError_t launch_status_min(unsigned long long* status, unsigned long long col, hipStream_t st) {
  k_status_min<<<1, 64, 0, st>>>(status, col);
  return hipGetLastError();
}

hipError_t launch_scatter_values(const DevSym& S, const double* vals, double* L, hipStream_t st) {
  if (S.nnzA <= 0) return hipSuccess;
  k_scatter_values<<<grid_for(S.nnzA), 256, 0, st>>>(S.amap, vals, S.nnzA, L);
  return hipGetLastError();
}

hipError_t launch_factor_panel(const DevSym& S, double* L, int64_t off, int32_t ntasks,
                               unsigned long long* status, double* winv, bool diag, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  if (diag) k_panel<<<ntasks, 256, 0, st>>>(S, L, off, status, winv);
  else k_panel_rows<<<ntasks, 256, 0, st>>>(S, L, off, winv);
  return hipGetLastError();
}

hipError_t launch_factor_la(const DevSym& S, double* L, int64_t off, int32_t nfirst, int32_t ntrsm, int32_t ntasks,
                            unsigned long long* status, double* winv, int32_t prec, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  const int32_t te = nfirst + ntrsm;
  if (prec == 2) k_panel_la<2><<<ntasks, 256, 0, st>>>(S, L, off, nfirst, te, status, winv);
  else if (prec == 1) k_panel_la<1><<<ntasks, 256, 0, st>>>(S, L, off, nfirst, te, status, winv);
  else k_panel_la<0><<<ntasks, 256, 0, st>>>(S, L, off, nfirst, te, status, winv);
  return hipGetLastError();
}

hipError_t launch_medium(const DevSym& S, double* L, int64_t off, int32_t nfirst, int32_t ntasks,
                         unsigned long long* status, double* winv, hipStream_t st) {
  if (nfirst > 0) k_medium<1><<<(nfirst + 3) / 4, 256, 0, st>>>(S, L, off, nfirst, status, winv);
  if (ntasks > nfirst)
    k_medium<2><<<(ntasks - nfirst + 3) / 4, 256, 0, st>>>(S, L, off + nfirst, ntasks - nfirst, status, winv);
  return hipGetLastError();
}

hipError_t launch_update_dense(const DevSym& S, double* L, int64_t off, int32_t ntasks, double* U, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  k_update<0, 5><<<ntasks, 256, 0, st>>>(S, L, off, U, 0);
  return hipGetLastError();
}

// Chunks of 64 tiles per XCD: at 64^3 the external update's L2 fetches per
// launch drop by a fifth against the plain round-robin order at the same
// speed; chunks of 256 or more leave XCDs unevenly loaded (slower).
constexpr int32_t kXcdGroup = 64;

hipError_t launch_update(const DevSym& S, double* L, int32_t kind, int64_t off, int32_t ntasks,
                         int32_t prec, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  const int32_t g = kXcdGroup;
  if (kind == 1) {
    if (prec == 2) k_update<2, 1><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else if (prec == 1) k_update<1, 1><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else k_update<0, 1><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
  } else if (kind == 4) {
    if (prec == 2) k_update<2, 4><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else if (prec == 1) k_update<1, 4><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else k_update<0, 4><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
  } else if (kind == 3) {
    if (prec == 2) k_update<2, 3><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else if (prec == 1) k_update<1, 3><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else k_update<0, 3><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
  } else {
    if (prec == 2) k_update<2, 2><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else if (prec == 1) k_update<1, 2><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
    else k_update<0, 2><<<ntasks, 256, 0, st>>>(S, L, off, nullptr, g);
  }
  return hipGetLastError();
}

hipError_t launch_small(const DevSym& S, double* L, int64_t off, int32_t ntasks, unsigned long long* status,
                        double* winv, int32_t prec, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  const int g = (ntasks + 3) / 4;
  if (prec == 2) k_small<2><<<g, 256, 0, st>>>(S, L, off, ntasks, status, winv);
  else if (prec == 1) k_small<1><<<g, 256, 0, st>>>(S, L, off, ntasks, status, winv);
  else k_small<0><<<g, 256, 0, st>>>(S, L, off, ntasks, status, winv);
  return hipGetLastError();
}

hipError_t launch_perm_gather(const DevSym& S, const double* B, int64_t ldb, int64_t nrhs, double* y,
                              hipStream_t st) {
  if (S.n * nrhs <= 0) return hipSuccess;
  k_perm_gather<<<grid_for(S.n * nrhs), 256, 0, st>>>(S.perm, S.n, B, ldb, nrhs, y);
  return hipGetLastError();
}

hipError_t launch_perm_scatter(const DevSym& S, const double* y, int64_t nrhs, double* B, int64_t ldb,
                               hipStream_t st) {
  if (S.n * nrhs <= 0) return hipSuccess;
  k_perm_scatter<<<grid_for(S.n * nrhs), 256, 0, st>>>(S.perm, S.n, y, nrhs, B, ldb);
  return hipGetLastError();
}

hipError_t launch_solve_step(const DevSym& S, const double* L, const double* winv, int32_t kind, int64_t off,
                             int32_t nfirst, int32_t ntasks, double* y, double* x, double* acc, int64_t nrhs,
                             hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  const int32_t n2 = ntasks - nfirst;  // (small kernels: supernodes with 65..128 rows below)
  if (kind == 3) k_fwd<<<ntasks, 256, 0, st>>>(S, L, winv, off, y, x, nrhs);
  else if (kind == 14) k_fwd2<<<ntasks, 256, 0, st>>>(S, L, winv, off, y, x, nrhs);
  else if (kind == 15) {
    if (nfirst > 0) k_fwd_small<false><<<(nfirst + 3) / 4, 256, 0, st>>>(S, L, winv, off, nfirst, y, x, nrhs);
    if (n2 > 0) k_fwd_small<true><<<(n2 + 3) / 4, 256, 0, st>>>(S, L, winv, off + nfirst, n2, y, x, nrhs);
  } else if (kind == 16) {
    if (nfirst > 0) k_bwd_small<false><<<(nfirst + 3) / 4, 256, 0, st>>>(S, L, winv, off, nfirst, x, nrhs);
    if (n2 > 0) k_bwd_small<true><<<(n2 + 3) / 4, 256, 0, st>>>(S, L, winv, off + nfirst, n2, x, nrhs);
  } else k_bwd<<<ntasks, 256, 0, st>>>(S, L, winv, off, x, acc, nrhs);
  return hipGetLastError();
}

int32_t logdet_partials(int64_t n) { return (int32_t)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

hipError_t launch_logdet(const DevSym& S, const double* L, double* partial, int32_t npartial, double* out,
                         hipStream_t st) {
  k_logdet_partial<<<npartial, 256, 0, st>>>(S, L, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_logdet_final<<<1, 256, 0, st>>>(partial, npartial, out);
  return hipGetLastError();
}

}  // namespace spchol

namespace spchol {

hipError_t launch_anorm(const DevSym& S, const double* vals, unsigned long long* out, hipStream_t st) {
  k_zero_u64<<<1, 64, 0, st>>>(out, 1);
  if (S.n > 0)
    k_anorm<<<(unsigned)std::min<int64_t>((S.n + 15) / 16, kStatBlocks), 256, 0, st>>>(S.a_rp, S.a_vidx, vals, S.n,
                                                                                      out);
  return hipGetLastError();
}

hipError_t launch_residual(const DevSym& S, const double* vals, const double* B, int64_t ldb, const double* X,
                           int64_t ldx, int64_t nrhs, double* R, unsigned long long* stats, hipStream_t st) {
  k_zero_u64<<<(unsigned)((3 * nrhs + 63) / 64), 64, 0, st>>>(stats, 3 * nrhs);
  if (S.n > 0)
    k_residual<<<(unsigned)std::min<int64_t>((S.n + 15) / 16, kStatBlocks), 256, 0, st>>>(S.a_rp, S.a_col, S.a_vidx, vals, S.n, B, ldb, X, ldx,
                                                            nrhs, R, stats);
  return hipGetLastError();
}

hipError_t launch_axpy(double* X, int64_t ldx, const double* D, int64_t n, int64_t nrhs, hipStream_t st) {
  if (n * nrhs <= 0) return hipSuccess;
  k_axpy<<<grid_for(n * nrhs), 256, 0, st>>>(X, ldx, D, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_dot_cols(const double* a, const double* b, int64_t n, int64_t nrhs, double* out,
                           hipStream_t st) {
  k_zero_u64<<<(unsigned)((nrhs + 63) / 64), 64, 0, st>>>(reinterpret_cast<unsigned long long*>(out), nrhs);
  if (n <= 0 || nrhs <= 0) return hipGetLastError();
  const int64_t per = std::min<int64_t>((n + 255) / 256, 512);
  k_dot_cols<<<dim3((unsigned)per, (unsigned)nrhs), 256, 0, st>>>(a, b, n, out);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(double* Y, int64_t ldy, const double* D, int64_t n, int64_t nrhs, const double* alpha,
                            hipStream_t st) {
  if (n * nrhs <= 0) return hipSuccess;
  k_axpy_cols<<<grid_for(n * nrhs), 256, 0, st>>>(Y, ldy, D, n, nrhs, alpha);
  return hipGetLastError();
}

hipError_t launch_xpby_cols(double* P, const double* Z, int64_t n, int64_t nrhs, const double* beta, hipStream_t st) {
  if (n * nrhs <= 0) return hipSuccess;
  k_xpby_cols<<<grid_for(n * nrhs), 256, 0, st>>>(P, Z, n, nrhs, beta);
  return hipGetLastError();
}

hipError_t launch_copy_cols(double* Y, int64_t ldy, const double* B, int64_t ldb, int64_t n, int64_t nrhs,
                            hipStream_t st) {
  if (n * nrhs <= 0) return hipSuccess;
  k_copy_cols<<<grid_for(n * nrhs), 256, 0, st>>>(Y, ldy, B, ldb, n, nrhs);
  return hipGetLastError();
}

}  // namespace spchol

namespace spchol {

hipError_t launch_si(const DevSym& S, int32_t kind, int64_t off, int32_t ntasks, const double* L, const double* winv,
                     double* Z, const int64_t* yoff, double* ybuf, double* tbuf, int32_t seglen, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  switch (kind) {
    case 9:
      if (seglen < 1 || seglen > kSiSeg) return hipErrorInvalidValue;
      k_si_y<<<ntasks, 256, 0, st>>>(S, L, Z, off, yoff, ybuf, seglen);
      break;
    case 10: k_si_zb<<<ntasks, 256, 0, st>>>(S, L, winv, Z, off, yoff, ybuf, tbuf); break;
    case 11: k_si_zd<<<ntasks, 256, 0, st>>>(S, winv, Z, off, tbuf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_abar(const DevSym& S, const double* Z, double g, const double* X, const double* lam, int64_t ld,
                       int64_t nrhs, double* Abar, hipStream_t st) {
  if (S.nnzA <= 0) return hipSuccess;
  k_abar<<<grid_for(S.nnzA), 256, 0, st>>>(S, Z, g, X, lam, ld, nrhs, Abar);
  return hipGetLastError();
}

}  // namespace spchol

namespace spchol {

// per-matrix logdet of a batch: one workgroup per matrix, columns of the
// matrix (permuted space keeps the blocks contiguous), tree reduction
__global__ __launch_bounds__(256) void k_logdet_segments(DevSym S, const double* __restrict__ L,
                                                         const int64_t* __restrict__ off, double* __restrict__ out) {
  __shared__ double sh[256];
  const int64_t b0 = off[blockIdx.x], b1 = off[blockIdx.x + 1];
  double v = 0.0;
  for (int64_t j = b0 + threadIdx.x; j < b1; j += 256) {
    const int J = S.snode_of[j];
    const int64_t d = j - S.sfirst[J];
    v += log(L[S.loff[J] + d * S.sm[J] + d]);
  }
  const double s = block_sum_256(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = 2.0 * s;
}

hipError_t launch_logdet_segments(const DevSym& S, const double* L, const int64_t* off, int32_t count, double* out,
                                  hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_logdet_segments<<<count, 256, 0, st>>>(S, L, off, out);
  return hipGetLastError();
}

}  // namespace spchol
