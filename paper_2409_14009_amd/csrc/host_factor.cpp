// Host side of the host-resident factorization (spchol_factor_streamed):
// the factor lives in host memory; supernodes below a size threshold are
// factored and applied to their ancestors by the host (the paper keeps
// small supernodes on the CPU, Sec. III), the others are factored on the
// GPU and their update matrices come back in column blocks that the host
// adds into the ancestors (the assembly of Sec. III, with the bounded
// update blocks of the second GPU-RLB version).
#include "host_factor.hpp"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

namespace spchol {

namespace {

// Run body(i) for i in [0, count) on up to `threads` threads (inline when
// the work is small).
template <class F>
void parallel_for(int64_t count, int threads, int64_t work_per_item, F&& body) {
  const int64_t grain = 1 << 16;  // at least this much work per thread
  int t = threads;
  if (t < 1) t = 1;
  const int64_t total = count * std::max<int64_t>(work_per_item, 1);
  if (t > 1 && total / grain < t) t = (int)std::max<int64_t>(1, total / grain);
  if (t <= 1 || count < 2) {
    for (int64_t i = 0; i < count; ++i) body(i);
    return;
  }
  std::vector<std::thread> pool;
  pool.reserve(t);
  for (int w = 0; w < t; ++w)
    pool.emplace_back([&, w] {
      for (int64_t i = w; i < count; i += t) body(i);  // interleaved: the columns' work shrinks with i
    });
  for (auto& th : pool) th.join();
}

}  // namespace

void host_scatter_values(const Symbolic& S, const double* vals, double* L) {
  std::fill(L, L + S.loff[S.ns], 0.0);
  for (int64_t p = 0; p < S.nnzA; ++p) L[S.amap[p]] = vals[p];
}

int64_t host_factor_supernode(const Symbolic& S, int64_t J, double* L) {
  const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
  double* B = L + S.loff[J];  // m x k, column-major, ld m
  // right-looking column Cholesky of the dense trapezoid (Sec. II-A: DPOTRF
  // of the diagonal block, then the rows below divided through)
  for (int64_t c = 0; c < k; ++c) {
    double* Lc = B + c * m;
    const double d = Lc[c];
    if (!(d > 0.0)) return S.sptr[J] + c;
    const double s = std::sqrt(d), inv = 1.0 / s;
    Lc[c] = s;
    for (int64_t i = c + 1; i < m; ++i) Lc[i] *= inv;
    for (int64_t c2 = c + 1; c2 < k; ++c2) {
      const double f = Lc[c2];
      if (f == 0.0) continue;
      double* L2 = B + c2 * m;
      for (int64_t i = c2; i < m; ++i) L2[i] -= Lc[i] * f;
    }
  }
  return -1;
}

void host_update_supernode(const Symbolic& S, int64_t J, double* L, int threads) {
  const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J], r = m - k;
  if (r <= 0) return;
  const double* B = L + S.loff[J];
  // rows below the diagonal block, row-major (contiguous dot products)
  std::vector<double> T((size_t)(r * k));
  for (int64_t t = 0; t < k; ++t)
    for (int64_t b = 0; b < r; ++b) T[b * k + t] = B[t * m + k + b];
  // column a of the update L_RJ L_RJ^T goes to one ancestor column (distinct
  // columns have distinct targets): parallel over a
  parallel_for(r, threads, (r / 2) * k, [&](int64_t a) {
    const int64_t o = S.obase[J] + a;
    const int64_t cbase = S.ocbase[o];
    const int64_t pr = S.opair[o];
    const int64_t a0 = S.pa0[pr], rel = S.relptr[pr];
    const double* Ta = T.data() + a * k;
    for (int64_t b = a; b < r; ++b) {
      const double* Tb = T.data() + b * k;
      double u = 0.0;
      for (int64_t t = 0; t < k; ++t) u += Tb[t] * Ta[t];
      L[cbase + S.tpos[rel + (b - a0)]] -= u;
    }
  });
}

void host_assemble_block(const Symbolic& S, int64_t J, int64_t cb, int64_t ce, const double* U, double* L,
                         int threads) {
  const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
  const int64_t ldu = m - cb;
  parallel_for(ce - cb, threads, (m - cb) / 2, [&](int64_t q) {
    const int64_t a = cb + q;  // local row of J = the update's column
    const int64_t o = S.obase[J] + (a - k);
    const int64_t cbase = S.ocbase[o];
    const int64_t pr = S.opair[o];
    const int64_t a0 = S.pa0[pr], rel = S.relptr[pr];
    const double* Uc = U + q * ldu;
    for (int64_t b = a; b < m; ++b) L[cbase + S.tpos[rel + (b - k - a0)]] -= Uc[b - cb];
  });
}

}  // namespace spchol
