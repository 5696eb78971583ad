// HIP kernels (gfx950) for the numeric phase of right-looking supernodal
// Cholesky (Sec. II-A), the supernodal triangular solves and logdet.
//
// Every launch processes a precomputed list of independent tasks (one
// workgroup each): the supernodes of one level of the supernodal
// elimination tree (Fig. 1), split into panels of at most 64 columns and
// 64-row tiles.  Storage: supernode J is a dense column-major m_J x k_J
// array (Sec. II-A), leading dimension m_J.
#include <climits>

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

// Columns of the block past kp are padded with an identity (unit
// diagonal, zero off-diagonal), so they factor to themselves and the sweep
// needs no per-column branch.  The pivot comes from its lane with readlane;
// the scaled column goes through LDS (colb, one wavefront) and is read back
// as a broadcast.  Like LAPACK's unblocked Cholesky, the column is scaled
// by the reciprocal of the pivot's square root.
__device__ __forceinline__ void potrf16(double (&r)[MB], int lane, int j0, double* __restrict__ colb,
                                        unsigned long long* __restrict__ status, int64_t col0) {
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    double piv = readlane_d(r[q], j0 + q);
    if (!(piv > 0.0)) {
      if (lane == j0 + q) atomicMin(status, (unsigned long long)(col0 + q));
      piv = 1.0;
    }
    const double ljj = sqrt(piv);
    const double rinv = 1.0 / ljj;
    const double lq = (lane == j0 + q) ? ljj : (lane > j0 + q ? r[q] * rinv : 0.0);
    r[q] = lq;
    colb[lane] = lq;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int c = q + 1; c < MB; ++c) r[c] = fma(-lq, colb[j0 + c], r[c]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// One wavefront's share of X = B W^T for a 64-row tile (B staged in LDS
// column-major As[k * DLD + r], W column-major Wc[c * DLD + i] = W_ic):
// wavefront w computes the 16 output columns 16w..16w+15 of all 64 rows on
// the fp64 matrix cores and writes them to rows R0.. of the panel.
__device__ __forceinline__ void trsm_tile_mfma(const double* __restrict__ As, const double* __restrict__ Wc,
                                               int kp, int lane, int w, double* __restrict__ Lp, int m,
                                               int R0) {
  if (MB * w >= kp) return;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  // k in chunks of 16: all LDS operands of a chunk are read before its
  // 16 MFMAs (columns past kp are zero in As)
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
  const int c = MB * w + li;
  if (c < kp) {
    double* dst = Lp + (int64_t)c * m;
#pragma unroll
    for (int rb2 = 0; rb2 < 4; ++rb2)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = R0 + 16 * rb2 + 4 * v + lk;
        if (r < m) dst[r] = acc[rb2][v];
      }
  }
}

// stage rows R0..R0+63 of the panel (kp columns) into As, zero padded
__device__ __forceinline__ void stage_rows(double* __restrict__ As, const double* __restrict__ Lp, int m, int kp,
                                           int R0, int tid, int nthr) {
  for (int base = 0; base < NBMAX * NBMAX; base += 16 * nthr) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * nthr + tid;
      const int r = idx & 63, c = idx >> 6;
      v[u] = (c < kp && R0 + r < m) ? Lp[(int64_t)c * m + R0 + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * nthr + tid;
      As[(idx >> 6) * DLD + (idx & 63)] = v[u];
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
//   4. when the panel has more rows (slot >= 0), W goes to scratch for the
//      row-tile launch.
__global__ __launch_bounds__(256) void k_panel(DevSym S, double* __restrict__ L, int64_t off,
                                               unsigned long long* __restrict__ status,
                                               double* __restrict__ scratch) {
  __shared__ __attribute__((aligned(16))) double Dc[NBMAX * DLD];
  __shared__ __attribute__((aligned(16))) double Wc[NBMAX * DLD];
  __shared__ __attribute__((aligned(16))) double colb[NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, rb = t.b, slot = t.c;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb;
  const int kp = min(S.nb, k - c0);
  const int nblk = (kp + MB - 1) / MB;
  double* __restrict__ Lp = L + S.loff[J] + (int64_t)c0 * m;  // Lp[c * m + r] = L[r, c0 + c]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  for (int base = 0; base < NBMAX * NBMAX; base += 16 * 256) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * 256 + tid;
      const int i = idx & 63, c = idx >> 6;
      const bool in = i < kp && c <= i;
      // clamped in-bounds address, value selected afterwards (no branch)
      const double x = Lp[(int64_t)min(c, kp - 1) * m + c0 + min(i, kp - 1)];
      v[u] = in ? x : (i == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * 256 + tid;
      Dc[(idx >> 6) * DLD + (idx & 63)] = v[u];
      Wc[(idx >> 6) * DLD + (idx & 63)] = 0.0;
    }
  }
  __syncthreads();

  // 1. Cholesky of the diagonal block, right-looking over 16-column blocks:
  //    wavefront 0 sweeps block column b (rows >= 16b), then the four
  //    wavefronts apply its update to the 16 x 16 blocks (i, b') with
  //    i >= b' > b on the matrix cores:
  //    D[i][b'] -= L[i][b] L[b'][b]^T
  for (int b = 0; b < nblk; ++b) {
    const int j0 = MB * b, jn = min(MB, kp - j0);
    const bool mine = (w == 0) && lane >= j0 && lane < kp;
    if (w == 0) {
      double xb[MB];
#pragma unroll
      for (int q = 0; q < MB; ++q) xb[q] = (lane >= j0) ? Dc[(j0 + q) * DLD + lane] : 0.0;
      // the sweep factors the 16 x 16 block (its lanes) and, on the lanes
      // below it, solves those rows against it
      potrf16(xb, lane, j0, colb, status, (int64_t)S.sfirst[J] + c0 + j0);
      if (mine) {
#pragma unroll
        for (int q = 0; q < MB; ++q)
          if (q < jn) Dc[(j0 + q) * DLD + lane] = (j0 + q <= lane) ? xb[q] : 0.0;
      }
    }
    __syncthreads();
    const int nrest = nblk - 1 - b;  // block columns right of b
    const int npairs = nrest * (nrest + 1) / 2;
    const int li = lane & 15, lk = lane >> 4;
    for (int pr = w; pr < npairs; pr += 4) {
      // pair index -> (i, bp) with b < bp <= i < nblk
      int bp = b + 1, rem = pr;
      while (rem >= nblk - bp) { rem -= nblk - bp; ++bp; }
      const int i = bp + rem;
      d4 P = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < MB; s += 4) {
        const double av = Dc[(j0 + s + lk) * DLD + MB * i + li];   // L[16i + li][16b + s + lk]
        const double bv = Dc[(j0 + s + lk) * DLD + MB * bp + li];  // L[16bp + li][16b + s + lk]
        P = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, P, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double* d = Dc + (MB * bp + li) * DLD + MB * i + 4 * v + lk;
        *d -= P[v];
      }
    }
    __syncthreads();
  }
  if (w == 0 && lane < kp) {
    double* dst = Lp + c0 + lane;
#pragma unroll 16
    for (int c = 0; c < NBMAX; ++c)
      if (c < kp && c <= lane) dst[(int64_t)c * m] = Dc[c * DLD + lane];
  }

  // 2a. inverses of the 16 x 16 diagonal blocks: lane l < 16 of wavefront w
  //     computes column l of inv(L_ww)
  if (w < nblk && lane < MB) {
    const int b0 = MB * w;
    double x[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      double s = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int q = 0; q < i; ++q) s = fma(-Dc[(b0 + q) * DLD + b0 + i], x[q], s);
      x[i] = s / Dc[(b0 + i) * DLD + b0 + i];
    }
#pragma unroll
    for (int i = 0; i < MB; ++i) Wc[(b0 + lane) * DLD + b0 + i] = x[i];
  }
  __syncthreads();
  // 2b. off-diagonal blocks of column block b = w, top to bottom
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
  __syncthreads();

  // 4. W for the row-tile launch, row-major: scratch[slot][r * 64 + c] = W_rc
  if (slot >= 0) {
    double* dst = scratch + (int64_t)slot * NBMAX * NBMAX;
    for (int idx = tid; idx < NBMAX * NBMAX; idx += 256) dst[idx] = Wc[(idx & 63) * DLD + (idx >> 6)];
  }
  // 3. rows rb .. rb + 255
  for (int R0 = rb; R0 < min(rb + 4 * 64, m); R0 += 64) {
    stage_rows(Dc, Lp, m, kp, R0, tid, 256);
    __syncthreads();
    trsm_tile_mfma(Dc, Wc, kp, lane, w, Lp, m, R0);
    __syncthreads();
  }
}

// Panel step, row tiles below the first 256 rows: X = B W^T with W from the
// scratch slot the diagonal task wrote (256 threads, one 64-row tile each).
__global__ __launch_bounds__(256) void k_panel_rows(DevSym S, double* __restrict__ L, int64_t off,
                                                    const double* __restrict__ scratch) {
  __shared__ __attribute__((aligned(16))) double As[NBMAX * DLD];
  __shared__ __attribute__((aligned(16))) double Wc[NBMAX * DLD];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, R0 = t.b, slot = t.c;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb;
  const int kp = min(S.nb, k - c0);
  double* __restrict__ Lp = L + S.loff[J] + (int64_t)c0 * m;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* src = scratch + (int64_t)slot * NBMAX * NBMAX;
  for (int base = 0; base < NBMAX * NBMAX; base += 16 * 256) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = src[base + u * 256 + tid];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = base + u * 256 + tid;  // idx = r * 64 + c
      Wc[(idx & 63) * DLD + (idx >> 6)] = v[u];
    }
  }
  stage_rows(As, Lp, m, kp, R0, tid, 256);
  __syncthreads();
  trsm_tile_mfma(As, Wc, kp, lane, w, Lp, m, R0);
}

// ---------------------------------------------------------------------------
// update: C[i, c] -= sum_t L[i, t] L[c, t] over a 64 x 64 tile, lower part,
// on the fp64 matrix cores (16x16x4 MFMA, four wavefronts of 32 x 32).
//   kind 1 (internal): the remaining columns of J itself, K = one panel;
//                      plain read-modify-write (one writer per entry).
//   kind 2 (external): the update matrix L_RJ L_RJ^T (Sec. II-A, Fig. 2),
//                      K = all columns of J, scattered into the ancestors
//                      through the relative indices; atomic adds because
//                      several supernodes of a level may hit one ancestor.
// MFMA operand layout (one wavefront, fp64 16x16x4, checked on gfx950):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[4 v + l / 16][l % 16] in its accumulator element v = 0..3.
// ---------------------------------------------------------------------------

constexpr int ALD = TILE + 2;

__global__ __launch_bounds__(256) void k_update(DevSym S, double* __restrict__ L, int32_t kind, int64_t off) {
  __shared__ double As[KC * ALD];
  __shared__ double Bs[KC * ALD];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, row0 = t.a, col0 = t.b;
  const int m = S.sm[J], k = S.sk[J];
  int kb, ke, colEnd;
  if (kind == 1) {
    kb = t.c * S.nb;
    ke = min(k, kb + S.nb);
    colEnd = k;
  } else {
    kb = 0;
    ke = k;
    colEnd = m;
  }
  double* __restrict__ Lj = L + S.loff[J];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // staging: thread loads rows (tid & 63) of chunk columns (tid >> 6) + 4q
  const int sr = tid & 63, sc = tid >> 6;
  const bool va = row0 + sr < m, vb = col0 + sr < colEnd;
  const double* pa = Lj + row0 + sr;
  const double* pb = Lj + col0 + sr;
  double ra[4], rb[4];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gc = kk + sc + 4 * q;
      ra[q] = (va && gc < ke) ? pa[(int64_t)gc * m] : 0.0;
      rb[q] = (vb && gc < ke) ? pb[(int64_t)gc * m] : 0.0;
    }
  };
  fetch(kb);
  for (int kk = kb; kk < ke; kk += KC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      As[(sc + 4 * q) * ALD + sr] = ra[q];
      Bs[(sc + 4 * q) * ALD + sr] = rb[q];
    }
    __syncthreads();
    if (kk + KC < ke) fetch(kk + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 4) {
      const int kr = (ks + lk) * ALD;
      const double a0 = As[kr + wr + li], a1 = As[kr + wr + 16 + li];
      const double b0 = Bs[kr + wc + li], b1 = Bs[kr + wc + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

  if (kind == 1) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int gc = col0 + wc + 16 * bj + li;
      if (gc >= colEnd) continue;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gr = row0 + wr + 16 * bi + 4 * v + lk;
          if (gr < m && gr >= gc) Lj[(int64_t)gc * m + gr] -= acc[bi][bj][v];
        }
    }
  } else {
    const int64_t ob = S.obase[J];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int gc = col0 + wc + 16 * bj + li;
      if (gc >= colEnd) continue;
      const int b = gc - k;
      const int pair = S.opair[ob + b];
      const int64_t cbase = S.ocbase[ob + b];
      const int32_t* __restrict__ tp = S.tpos + S.relptr[pair] - S.pa0[pair] - k;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gr = row0 + wr + 16 * bi + 4 * v + lk;
          if (gr < m && gr >= gc) atomicAdd(L + cbase + tp[gr], -acc[bi][bj][v]);
        }
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
__global__ __launch_bounds__(64) void k_fwd_tri(DevSym S, const double* __restrict__ L, int64_t off,
                                                double* __restrict__ y, int64_t nrhs) {
  __shared__ double Dc[NBMAX * DLD];  // column-major: Dc[c * DLD + i] = D_ic
  __shared__ double rinv[NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ src = L + S.loff[J] + (int64_t)c0 * m + c0;
  const int lane = threadIdx.x;
  for (int cb = 0; cb < kp; cb += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int c = cb + u;
      v[u] = (c < kp && lane < kp && c <= lane) ? src[(int64_t)c * m + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) Dc[(cb + u) * DLD + lane] = v[u];
  }
  __syncthreads();
  if (lane < kp) rinv[lane] = 1.0 / Dc[lane * DLD + lane];
  __syncthreads();
  const int64_t g = S.sfirst[J] + c0 + lane;
  for (int64_t c = 0; c < nrhs; ++c) {
    double v = lane < kp ? y[g + c * S.n] : 0.0;
    for (int j = 0; j < kp; ++j) {
      const double vj = readlane_d(v, j) * rinv[j];
      if (lane == j) v = vj;
      else if (lane > j) v = fma(-Dc[j * DLD + lane], vj, v);
    }
    if (lane < kp) y[g + c * S.n] = v;
  }
}

// forward: y[rows below the panel] -= L[rows, panel] y_p
__global__ __launch_bounds__(256) void k_fwd_gemv(DevSym S, const double* __restrict__ L, int64_t off,
                                                  double* __restrict__ y, int64_t nrhs) {
  __shared__ double yp[NBMAX][4];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, r0 = t.b;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  const int64_t first = S.sfirst[J];
  const int tid = threadIdx.x;
  const int row = r0 + (tid % 64);
  const int cs = tid / 64;
  for (int64_t cb = 0; cb < nrhs; cb += 4) {
    __syncthreads();
    for (int idx = tid; idx < kp * 4; idx += 256) {
      const int tt = idx % kp, cc = idx / kp;
      yp[tt][cc] = (cb + cc < nrhs) ? y[first + c0 + tt + (cb + cc) * S.n] : 0.0;
    }
    __syncthreads();
    const int64_t c = cb + cs;
    if (row < m && c < nrhs) {
      double s = 0.0;
      for (int tt = 0; tt < kp; ++tt) s = fma(Lj[(int64_t)(c0 + tt) * m + row], yp[tt][cs], s);
      double* dst = y + R[row] + c * S.n;
      if (row < k) *dst -= s;
      else atomicAdd(dst, -s);
    }
  }
}

// backward: y_p -= L[rows below, panel]^T y[rows below]
__global__ __launch_bounds__(256) void k_bwd_gemvt(DevSym S, const double* __restrict__ L, int64_t off,
                                                   double* __restrict__ y, int64_t nrhs) {
  __shared__ double Ls[TILE][NBMAX + 1];
  __shared__ double ys[TILE];
  __shared__ double red[4][NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, r0 = t.b;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const int32_t* __restrict__ R = S.rows + S.rptr[J];
  const int64_t first = S.sfirst[J];
  const int tid = threadIdx.x;
  const int nr = min(TILE, m - r0);
  for (int idx = tid; idx < nr * kp; idx += 256) {
    const int r = idx % nr, tt = idx / nr;
    Ls[r][tt] = Lj[(int64_t)(c0 + tt) * m + r0 + r];
  }
  const int tt = tid % 64, rg = tid / 64;
  for (int64_t c = 0; c < nrhs; ++c) {
    __syncthreads();
    for (int r = tid; r < nr; r += 256) ys[r] = y[R[r0 + r] + c * S.n];
    __syncthreads();
    double s = 0.0;
    if (tt < kp) {
      const int rend = min(nr, rg * 16 + 16);
      for (int r = rg * 16; r < rend; ++r) s = fma(Ls[r][tt], ys[r], s);
    }
    red[rg][tt] = s;
    __syncthreads();
    if (tid < kp) {
      const double v = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
      atomicAdd(y + first + c0 + tid + c * S.n, -v);
    }
  }
}

// backward: y_p <- D_p^{-T} y_p; row sweep from the bottom, the block kept
// row-major (Dr[j * DLD + i] = D_ji) so lane i reads D_ji contiguously
__global__ __launch_bounds__(64) void k_bwd_tri(DevSym S, const double* __restrict__ L, int64_t off,
                                                double* __restrict__ y, int64_t nrhs) {
  __shared__ double Dr[NBMAX * DLD];
  __shared__ double rinv[NBMAX];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ src = L + S.loff[J] + (int64_t)c0 * m + c0;
  const int lane = threadIdx.x;
  for (int ib = 0; ib < kp; ib += 16) {  // lane = row j of the block, column i
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = ib + u;
      v[u] = (i < kp && lane < kp && i <= lane) ? src[(int64_t)i * m + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) Dr[lane * DLD + ib + u] = v[u];
  }
  __syncthreads();
  if (lane < kp) rinv[lane] = 1.0 / Dr[lane * DLD + lane];
  __syncthreads();
  const int64_t g = S.sfirst[J] + c0 + lane;
  for (int64_t c = 0; c < nrhs; ++c) {
    double v = lane < kp ? y[g + c * S.n] : 0.0;
    for (int j = kp - 1; j >= 0; --j) {
      const double vj = readlane_d(v, j) * rinv[j];
      if (lane == j) v = vj;
      else if (lane < j) v = fma(-Dr[j * DLD + lane], vj, v);
    }
    if (lane < kp) y[g + c * S.n] = v;
  }
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

hipError_t launch_scatter_values(const DevSym& S, const double* vals, double* L, hipStream_t st) {
  if (S.nnzA <= 0) return hipSuccess;
  k_scatter_values<<<grid_for(S.nnzA), 256, 0, st>>>(S.amap, vals, S.nnzA, L);
  return hipGetLastError();
}

hipError_t launch_factor_panel(const DevSym& S, double* L, int64_t off, int32_t ntasks,
                               unsigned long long* status, double* scratch, bool diag, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  if (diag) k_panel<<<ntasks, 256, 0, st>>>(S, L, off, status, scratch);
  else k_panel_rows<<<ntasks, 256, 0, st>>>(S, L, off, scratch);
  return hipGetLastError();
}

hipError_t launch_update(const DevSym& S, double* L, int32_t kind, int64_t off, int32_t ntasks,
                         hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  k_update<<<ntasks, 256, 0, st>>>(S, L, kind, off);
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

hipError_t launch_solve_step(const DevSym& S, const double* L, int32_t kind, int64_t off, int32_t ntasks,
                             double* y, int64_t nrhs, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  switch (kind) {
    case 3: k_fwd_tri<<<ntasks, 64, 0, st>>>(S, L, off, y, nrhs); break;
    case 4: k_fwd_gemv<<<ntasks, 256, 0, st>>>(S, L, off, y, nrhs); break;
    case 5: k_bwd_gemvt<<<ntasks, 256, 0, st>>>(S, L, off, y, nrhs); break;
    case 6: k_bwd_tri<<<ntasks, 64, 0, st>>>(S, L, off, y, nrhs); break;
    default: return hipErrorInvalidValue;
  }
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
