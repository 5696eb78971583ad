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
// panel factorization: Cholesky of the diagonal block + triangular solve of
// one 64-row tile of the panel (Sec. II-A: DPOTRF then DTRSM).  Every tile
// factors the small diagonal block itself in LDS; the tile that contains
// it writes it back and reports a non-positive pivot.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_factor_panel(DevSym S, double* __restrict__ L, int64_t off,
                                                      unsigned long long* __restrict__ status) {
  __shared__ double D[NBMAX][NBMAX + 1];
  __shared__ double X[TILE][NBMAX + 1];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a, row0 = t.b;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb;
  const int kp = min(S.nb, k - c0);
  double* __restrict__ Lj = L + S.loff[J];
  const int tid = threadIdx.x;
  const bool diag_tile = (row0 == c0);

  for (int idx = tid; idx < kp * kp; idx += 256) {
    const int i = idx % kp, j = idx / kp;
    D[i][j] = (i >= j) ? Lj[(int64_t)(c0 + j) * m + c0 + i] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kp; ++j) {
    if (tid == 0) {
      double d = D[j][j];
      if (!(d > 0.0)) {
        if (diag_tile) atomicMin(status, (unsigned long long)(S.sfirst[J] + c0 + j));
        d = 1.0;
      }
      D[j][j] = sqrt(d);
    }
    __syncthreads();
    const double djj = D[j][j];
    for (int i = j + 1 + tid; i < kp; i += 256) D[i][j] /= djj;
    __syncthreads();
    const int nt = kp - j - 1;
    for (int idx = tid; idx < nt * nt; idx += 256) {
      const int i = j + 1 + idx % nt, c = j + 1 + idx / nt;
      if (i >= c) D[i][c] -= D[i][j] * D[c][j];
    }
    __syncthreads();
  }

  // rows of this tile that need the triangular solve
  const int rb = diag_tile ? c0 + kp : row0;
  const int re = min(row0 + TILE, m);
  const int nr = re - rb;
  if (nr > 0) {
    for (int idx = tid; idx < nr * kp; idx += 256) {
      const int r = idx % nr, j = idx / nr;
      X[r][j] = Lj[(int64_t)(c0 + j) * m + rb + r];
    }
    __syncthreads();
    for (int j = 0; j < kp; ++j) {
      const double djj = D[j][j];
      for (int r = tid; r < nr; r += 256) X[r][j] /= djj;
      __syncthreads();
      const int nc = kp - j - 1;
      for (int idx = tid; idx < nr * nc; idx += 256) {
        const int r = idx % nr, c = j + 1 + idx / nr;
        X[r][c] -= X[r][j] * D[c][j];
      }
      __syncthreads();
    }
    for (int idx = tid; idx < nr * kp; idx += 256) {
      const int r = idx % nr, j = idx / nr;
      Lj[(int64_t)(c0 + j) * m + rb + r] = X[r][j];
    }
  }
  if (diag_tile) {
    for (int idx = tid; idx < kp * kp; idx += 256) {
      const int i = idx % kp, j = idx / kp;
      if (i >= j) Lj[(int64_t)(c0 + j) * m + c0 + i] = D[i][j];
    }
  }
}

// ---------------------------------------------------------------------------
// update: C[i, c] -= sum_t L[i, t] L[c, t] over a 64 x 64 tile, lower part.
//   kind 1 (internal): the remaining columns of J itself, K = one panel;
//                      plain read-modify-write (one writer per entry).
//   kind 2 (external): the update matrix L_RJ L_RJ^T (Sec. II-A, Fig. 2),
//                      K = all columns of J, scattered into the ancestors
//                      through the relative indices; atomic adds because
//                      several supernodes of a level may hit one ancestor.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_update(DevSym S, double* __restrict__ L, int32_t kind, int64_t off) {
  __shared__ double As[KC][TILE + 1];
  __shared__ double Bs[KC][TILE + 1];
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
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

  for (int kk = kb; kk < ke; kk += KC) {
    for (int idx = tid; idx < TILE * KC; idx += 256) {
      const int r = idx % TILE, c = idx / TILE;
      const int gc = kk + c;
      const int ga = row0 + r, gb = col0 + r;
      As[c][r] = (ga < m && gc < ke) ? Lj[(int64_t)gc * m + ga] : 0.0;
      Bs[c][r] = (gb < colEnd && gc < ke) ? Lj[(int64_t)gc * m + gb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[c][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[c][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

  if (kind == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + ty + 16 * j;
      if (gc >= colEnd) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = row0 + tx + 16 * i;
        if (gr < m && gr >= gc) Lj[(int64_t)gc * m + gr] -= acc[i][j];
      }
    }
  } else {
    const int64_t ob = S.obase[J];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gc = col0 + ty + 16 * j;
      if (gc >= colEnd) continue;
      const int b = gc - k;
      const int pair = S.opair[ob + b];
      const int64_t cbase = S.ocbase[ob + b];
      const int32_t* __restrict__ tp = S.tpos + S.relptr[pair] - S.pa0[pair];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gr = row0 + tx + 16 * i;
        if (gr < m && gr >= gc) atomicAdd(L + cbase + tp[gr - k], -acc[i][j]);
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

__device__ inline void load_diag_block(double (*D)[NBMAX + 1], const double* __restrict__ Lj, int m, int c0,
                                       int kp, int tid, int nthreads) {
  for (int idx = tid; idx < kp * kp; idx += nthreads) {
    const int i = idx % kp, j = idx / kp;
    D[i][j] = (i >= j) ? Lj[(int64_t)(c0 + j) * m + c0 + i] : 0.0;
  }
}

// forward: y_p <- D_p^{-1} y_p, one wavefront per (J, panel)
__global__ __launch_bounds__(64) void k_fwd_tri(DevSym S, const double* __restrict__ L, int64_t off,
                                                double* __restrict__ y, int64_t nrhs) {
  __shared__ double D[NBMAX][NBMAX + 1];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const int lane = threadIdx.x;
  load_diag_block(D, Lj, m, c0, kp, lane, 64);
  __syncthreads();
  const int64_t g = S.sfirst[J] + c0 + lane;
  for (int64_t c = 0; c < nrhs; ++c) {
    double v = lane < kp ? y[g + c * S.n] : 0.0;
    for (int j = 0; j < kp; ++j) {
      const double vj = __shfl(v, j) / D[j][j];
      if (lane == j) v = vj;
      else if (lane > j && lane < kp) v -= D[lane][j] * vj;
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

// backward: y_p <- D_p^{-T} y_p
__global__ __launch_bounds__(64) void k_bwd_tri(DevSym S, const double* __restrict__ L, int64_t off,
                                                double* __restrict__ y, int64_t nrhs) {
  __shared__ double D[NBMAX][NBMAX + 1];
  const DevTask t = S.tasks[off + blockIdx.x];
  const int J = t.J, p = t.a;
  const int m = S.sm[J], k = S.sk[J];
  const int c0 = p * S.nb, kp = min(S.nb, k - c0);
  const double* __restrict__ Lj = L + S.loff[J];
  const int lane = threadIdx.x;
  load_diag_block(D, Lj, m, c0, kp, lane, 64);
  __syncthreads();
  const int64_t g = S.sfirst[J] + c0 + lane;
  for (int64_t c = 0; c < nrhs; ++c) {
    double v = lane < kp ? y[g + c * S.n] : 0.0;
    for (int j = kp - 1; j >= 0; --j) {
      const double vj = __shfl(v, j) / D[j][j];
      if (lane == j) v = vj;
      else if (lane < j) v -= D[j][lane] * vj;
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
                               unsigned long long* status, hipStream_t st) {
  if (ntasks <= 0) return hipSuccess;
  k_factor_panel<<<ntasks, 256, 0, st>>>(S, L, off, status);
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
