// Device-side view of the symbolic analysis and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace spchol {

struct DevTask {
  int32_t J, a, b, c;
};

// All arrays live in device memory; passed to kernels by value.
struct DevSym {
  const int64_t* loff;    // ns+1 storage offsets (doubles)
  const int32_t* sk;      // ns: columns k_J
  const int32_t* sm;      // ns: rows m_J
  const int32_t* sfirst;  // ns: first column
  const int64_t* rptr;    // ns+1 row-list offsets
  const int32_t* rows;    // row lists (permuted global indices)
  const int64_t* obase;   // ns+1 offsets of per-off-diagonal-row arrays
  const int32_t* opair;   // pair id of each off-diagonal row
  const int64_t* ocbase;  // storage offset of the target column of each off-diagonal row
  const int32_t* pa0;     // npairs: first off-diagonal row of J inside P
  const int64_t* relptr;  // npairs+1
  const int32_t* tpos;    // position from the top of the row in P's row list
  const int32_t* snode_of;// n
  const int64_t* amap;    // nnzA
  const int64_t* perm;    // n
  const DevTask* tasks;
  const int64_t* a_rp;    // n+1: full-symmetric CSR of A (original ordering)
  const int32_t* a_col;   // column of each entry
  const int64_t* a_vidx;  // index of each entry in the stored lower values
  const int32_t* e_row;   // nnzA: row of each stored lower entry of A (original)
  const int32_t* e_col;   // nnzA: its column
  const int64_t* wbase;   // ns+1: offsets of the panels' inverted diagonal blocks
  int64_t n, ns, nnzA, storage;
  int32_t nb;
};

// launchers (kernels.hip); all enqueue on `st` and return hipGetLastError()
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t st);
hipError_t launch_status_init(unsigned long long* status, hipStream_t st);
hipError_t launch_status_min(unsigned long long* status, unsigned long long col, hipStream_t st);
hipError_t launch_scatter_values(const DevSym& S, const double* vals, double* L, hipStream_t st);
hipError_t launch_factor_panel(const DevSym& S, double* L, int64_t off, int32_t ntasks,
                               unsigned long long* status, double* winv, bool diag, hipStream_t st);
// kind 1: internal tiles (plain read-modify-write); 2: external tiles,
// fp64 atomic adds; 3: external tiles, plain read-modify-write (only for
// launches whose tasks add into disjoint entries); 4: RLB block-pair tiles,
// fp64 atomic adds at addresses from one relative index per block
hipError_t launch_update(const DevSym& S, double* L, int32_t kind, int64_t off, int32_t ntasks,
                         int32_t prec, hipStream_t st);
// update tiles (J, first local row, first local col, cb) of a column block
// cb.. of L_RJ L_RJ^T written to U (column-major, leading dimension m_J - cb,
// lower part; fp64), not scattered: the host-resident factorization
// one-panel supernodes of at most 32 columns, one wavefront each: factor,
// inverse block, all rows below (no update); tasks [0, nfirst) have at most
// 16 columns, the rest 17 to 32
hipError_t launch_medium(const DevSym& S, double* L, int64_t off, int32_t nfirst, int32_t ntasks,
                         unsigned long long* status, double* winv, hipStream_t st);
hipError_t launch_update_dense(const DevSym& S, double* L, int64_t off, int32_t ntasks, double* U, hipStream_t st);
// tasks [0, nfirst): diagonal tasks; then ntrsm row tiles; the rest internal
// update tiles
hipError_t launch_factor_la(const DevSym& S, double* L, int64_t off, int32_t nfirst, int32_t ntrsm, int32_t ntasks,
                            unsigned long long* status, double* winv, int32_t prec, hipStream_t st);
hipError_t launch_si(const DevSym& S, int32_t kind, int64_t off, int32_t ntasks, const double* L, const double* winv,
                     double* Z, const int64_t* yoff, double* ybuf, double* tbuf, int32_t seglen, hipStream_t st);
hipError_t launch_abar(const DevSym& S, const double* Z, double g, const double* X, const double* lam, int64_t ld,
                       int64_t nrhs, double* Abar, hipStream_t st);
hipError_t launch_anorm(const DevSym& S, const double* vals, unsigned long long* out, hipStream_t st);
hipError_t launch_residual(const DevSym& S, const double* vals, const double* B, int64_t ldb, const double* X,
                           int64_t ldx, int64_t nrhs, double* R, unsigned long long* stats, hipStream_t st);
hipError_t launch_axpy(double* X, int64_t ldx, const double* D, int64_t n, int64_t nrhs, hipStream_t st);
// preconditioned conjugate gradients: out[c] = a[:, c] . b[:, c];
// Y[:, c] += alpha[c] D[:, c]; P[:, c] = Z[:, c] + beta[c] P[:, c]
// (blocks n x nrhs with leading dimension n, except Y: ldy; scalars on the
// device).  launch_residual with B == NULL gives R = -A X.
hipError_t launch_dot_cols(const double* a, const double* b, int64_t n, int64_t nrhs, double* out, hipStream_t st);
hipError_t launch_axpy_cols(double* Y, int64_t ldy, const double* D, int64_t n, int64_t nrhs, const double* alpha,
                            hipStream_t st);
hipError_t launch_xpby_cols(double* P, const double* Z, int64_t n, int64_t nrhs, const double* beta, hipStream_t st);
hipError_t launch_copy_cols(double* Y, int64_t ldy, const double* B, int64_t ldb, int64_t n, int64_t nrhs,
                            hipStream_t st);
// one wavefront per supernode of a K_SMALL launch (four per workgroup);
// prec as for launch_update (the precision of the update products)
hipError_t launch_small(const DevSym& S, double* L, int64_t off, int32_t ntasks, unsigned long long* status,
                        double* winv, int32_t prec, hipStream_t st);
hipError_t launch_perm_gather(const DevSym& S, const double* B, int64_t ldb, int64_t nrhs, double* y,
                              hipStream_t st);
hipError_t launch_perm_scatter(const DevSym& S, const double* y, int64_t nrhs, double* B, int64_t ldb,
                               hipStream_t st);
// one solve launch of the plans; nfirst: for the small-supernode kinds, the
// leading tasks with at most 64 rows below (a kernel without the second
// row chunk), the rest with 65 to 128
hipError_t launch_solve_step(const DevSym& S, const double* L, const double* winv, int32_t kind, int64_t off,
                             int32_t nfirst, int32_t ntasks, double* y, double* x, double* acc, int64_t nrhs,
                             hipStream_t st);
hipError_t launch_logdet(const DevSym& S, const double* L, double* partial, int32_t npartial,
                         double* out, hipStream_t st);
int32_t logdet_partials(int64_t n);
hipError_t launch_logdet_segments(const DevSym& S, const double* L, const int64_t* off, int32_t count, double* out,
                                  hipStream_t st);

}  // namespace spchol
