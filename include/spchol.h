/*
 * spchol.h -- C ABI of an MI355X (gfx950) supernodal sparse Cholesky library.
 *
 * The method is the right-looking supernodal factorization of a sparse
 * symmetric positive definite matrix A = L L^T (Sec. II of "GPU Accelerated
 * Sparse Cholesky Factorization", Karsavuran, Ng and Peyton): for every
 * supernode J, leaves to root, a dense Cholesky of its diagonal block, a
 * triangular solve of its off-diagonal panel, then the update L_RJ L_RJ^T
 * scattered through relative indices into the ancestor supernodes it touches
 * (Sec. II-A, Fig. 2).  The triangular solves (Sec. I) and the
 * log-determinant follow.  All numeric work runs in HIP kernels on one GPU;
 * the factor stays resident in device memory.
 *
 * Conventions for every entry point
 *  - Indices are 0-based.  A matrix is given by its lower triangle, diagonal
 *    included, in compressed-column form: colptr[n+1], rowind[colptr[n]],
 *    rows strictly increasing inside each column, every row >= its column,
 *    every diagonal entry present.  vals follow rowind's order.
 *  - perm[k] is the original index eliminated k-th (NULL = identity).  The
 *    factor is that of C = P A P^T with C_kk' = A_{perm[k], perm[k']}.
 *  - "host" pointers are read during the call only.  "device" pointers are
 *    hipMalloc'ed (coarse-grained) device memory owned by the caller; they
 *    must stay valid until the work enqueued on `stream` has completed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it; only the calls that return a
 *    host value (spchol_factor's info, spchol_logdet) synchronize it.
 *  - Handles are owned by the library and freed with their destroy call.
 *    A spchol_num keeps a reference to its spchol_sym: destroy the num
 *    first.  Handles may be used from one host thread at a time.  A
 *    spchol_num owns a second stream (factorization: external updates
 *    beside the next level's panels; solves: every other group of four
 *    right-hand sides) that waits for the caller's stream and is joined
 *    back into it within each call, and its workspaces: work enqueued with
 *    one num on two streams at once must be ordered by the caller.
 *  - On error the status is negative, outputs are unspecified, handles stay
 *    valid and spchol_last_error() returns a message (thread-local).
 *  - No C++ exception crosses this boundary.
 */
#ifndef SPCHOL_H
#define SPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spchol_sym_s *spchol_sym; /* symbolic analysis (host + device copy) */
typedef struct spchol_num_s *spchol_num; /* numeric factor (device memory)        */
typedef struct spchol_graph_s *spchol_graph; /* captured factor (+ solve) launch sequence */

typedef enum {
  SPCHOL_OK = 0,
  SPCHOL_ERR_ARG = -1,     /* null or inconsistent argument               */
  SPCHOL_ERR_PATTERN = -2, /* unsorted/duplicate/upper entry, no diagonal */
  SPCHOL_ERR_NOT_SPD = -3, /* a pivot was not positive (see info)         */
  SPCHOL_ERR_OOM = -4,     /* host or device allocation failed            */
  SPCHOL_ERR_HIP = -5,     /* a HIP runtime call failed                   */
  SPCHOL_ERR_NOCONV = -6   /* iterative refinement did not converge       */
} spchol_status;

/* Supernode partition (Sec. I: columns with the same structure form a
 * dense submatrix).  FUNDAMENTAL: column j+1 joins j's supernode when j is
 * its only etree child and struct(L_j) \ {j} = struct(L_{j+1}).  MAXIMAL:
 * the only-child condition is dropped (the partition drawn in Fig. 1). */
enum { SPCHOL_SNODE_FUNDAMENTAL = 0, SPCHOL_SNODE_MAXIMAL = 1 };

typedef struct {
  int32_t snode_mode;      /* SPCHOL_SNODE_*                                    */
  int32_t amalg_max_zeros; /* relaxed amalgamation (Sec. IV-A merges a supernode
                              with its parent): a supernode is merged into its
                              parent when the parent's columns follow right after
                              its own and the merged dense storage holds at most
                              this many explicit zeros per column; 0 = off      */
  int32_t panel_width;     /* columns per factorization panel (0 = default 64,
                              must be a multiple of 16 and <= 64)              */
  int32_t deterministic;   /* nonzero: bitwise reproducible factorization,
                              solves and selected inversion.  Concurrent
                              supernodes add into shared ancestor entries
                              (Sec. II-A) with fp64 atomics, whose order, and
                              so the last bits, vary between runs; this mode
                              splits every such launch into launches whose
                              adds hit disjoint entries (a colouring of each
                              level's supernodes by shared rows), run in a
                              fixed order, never splits a backward-solve
                              panel, and runs no update beside the next
                              level.  More launches, same arithmetic.  The
                              environment variable SPCHOL_DETERMINISTIC=1
                              forces it at analysis.                         */
  int64_t workspace_limit; /* bytes of device memory a numeric handle may
                              hold (factor, inverse blocks, the analysis'
                              device copy, solve / refinement / selected-
                              inversion workspaces); 0 = no limit.  A call
                              that would exceed it fails with SPCHOL_ERR_OOM
                              before allocating or enqueuing anything.       */
  int32_t amalg_rule;      /* SPCHOL_AMALG_*: how supernodes are merged      */
  int32_t amalg_cap_percent; /* SPCHOL_AMALG_GREEDY: largest increase of the
                              factor's storage, percent of nnz(L) (25)        */
  int32_t update_method;   /* SPCHOL_UPDATE_*: how a supernode's update
                              reaches its ancestors                          */
  int32_t partition_refinement; /* nonzero: reorder the columns inside each
                              (unmerged) supernode so that the rows of its
                              descendants form fewer, longer runs of
                              consecutive indices (Sec. IV-A; same fill).
                              The elimination order then differs from perm:
                              spchol_sym_perm returns the one used.          */
} spchol_options;

/* Update methods.  RL (Sec. II-A): the update L_RJ L_RJ^T in 64 x 64 tiles,
 * each entry added into its ancestor through the relative index of its row.
 * RLB (Sec. II-B): J's rows below its columns form blocks of consecutive
 * indices inside one ancestor; every pair of blocks (B below or equal B')
 * is a product added straight into the ancestor's storage, addressed by one
 * relative index per block (tiles of at most 64 x 64 inside each pair). */
enum { SPCHOL_UPDATE_RL = 0, SPCHOL_UPDATE_RLB = 1 };

/* Amalgamation rules.  ZEROS: visit supernodes by first column, merge each
 * into its parent when the parent's columns follow right after it and the
 * merged dense storage holds at most amalg_max_zeros explicit zeros per
 * column (0 = no merging).  GREEDY (Sec. IV-A): merge pairs (J, p(J)) in
 * sequence, each step the pair adding the least new fill (explicit zeros of
 * the merged trapezoid), ties to the smaller first column, until the
 * cumulative increase would pass amalg_cap_percent of nnz(L); only pairs
 * whose columns are consecutive qualify (the ordering is the caller's). */
enum { SPCHOL_AMALG_ZEROS = 0, SPCHOL_AMALG_GREEDY = 1 };

/* Fill *opt with the defaults (fundamental, no amalgamation (ZEROS rule,
 * 0 zeros; GREEDY cap 25 %), panel 64, atomic scatter, no workspace
 * limit). */
spchol_status spchol_default_options(spchol_options *opt);

/* Fill-reducing ordering of a general sparse symmetric pattern (host only):
 * nested dissection by multilevel graph bisection, this library's stand-in
 * for the METIS ordering of Sec. IV-A.  Coarsening by heavy-edge matching,
 * bisection of the coarsest graph by greedy growing, Fiduccia-Mattheyses
 * refinement while projecting back, a minimum vertex cover of the cut edges
 * as the separator; parts of at most leaf_size vertices (0 = 64) ordered by
 * minimum degree.  Same result for the same seed.
 *   n, colptr, rowind: host, CSC pattern (lower triangle as in
 *     spchol_analyze, or both triangles; the diagonal is ignored);
 *   perm_out: host, n entries: perm_out[k] = the original index eliminated
 *     k-th, ready to pass to spchol_analyze.
 * Errors: SPCHOL_ERR_ARG, SPCHOL_ERR_PATTERN (row out of range),
 * SPCHOL_ERR_OOM. */
spchol_status spchol_order_nd(int64_t n, const int64_t *colptr, const int64_t *rowind, int64_t leaf_size,
                              uint64_t seed, int64_t *perm_out);

/* Symbolic analysis (host only, no device work): elimination tree (Sec. II),
 * column counts, supernode partition and amalgamation, supernodal elimination
 * tree (Fig. 1), row lists, relative indices relind(J, P) (Sec. II-A), the map
 * from A's entries to factor storage, and the leaves-to-root level schedule.
 *   n, colptr, rowind: host, lower CSC pattern of A (see conventions).
 *   perm: host, n entries or NULL.
 *   opt: host or NULL (defaults).
 *   out: receives a new handle.
 * Errors: SPCHOL_ERR_ARG (n < 0, null pointer, perm not a permutation),
 * SPCHOL_ERR_PATTERN (pattern violates the conventions), SPCHOL_ERR_OOM. */
spchol_status spchol_analyze(int64_t n, const int64_t *colptr, const int64_t *rowind,
                             const int64_t *perm, const spchol_options *opt, spchol_sym *out);

/* Batch of independent matrices analysed as one block-diagonal matrix (a
 * forest of elimination trees): every level launch of the factorization,
 * the solves and the reverse mode then covers the supernodes of all the
 * matrices at once.  Matrix b occupies columns col_off[b]..col_off[b+1]-1
 * (in both the original and the permuted numbering) and stored entries
 * nz_off[b].. of the concatenated value array.  Arrays as in
 * spchol_analyze, one per matrix (host); perm may be NULL or hold NULLs. */
spchol_status spchol_batch_analyze(int32_t count, const int64_t *n, const int64_t *const *colptr,
                                   const int64_t *const *rowind, const int64_t *const *perm,
                                   const spchol_options *opt, spchol_sym *out);

/* Batch layout (host outputs, may be NULL): count; col_off[count+1];
 * nz_off[count+1].  A handle from spchol_analyze reports one matrix. */
spchol_status spchol_batch_info(spchol_sym sym, int32_t *count, int64_t *col_off, int64_t *nz_off);

/* The elimination order of the analysis (host output, n entries): perm
 * as given, or the refined order when partition_refinement was set; the
 * factor is that of C = P A P^T for this order. */
spchol_status spchol_sym_perm(spchol_sym sym, int64_t *perm_out);

/* Summary of a symbolic analysis (host output). */
typedef struct {
  int64_t n;
  int64_t nnz_a;        /* stored lower entries of A                          */
  int64_t nnz_l;        /* true nonzeros of L (sum of column counts)         */
  int64_t storage;      /* doubles of supernodal storage (sum m_J * k_J)     */
  int64_t nsuper;       /* supernodes after amalgamation                      */
  int64_t nrows_total;  /* sum of supernode row-list lengths m_J              */
  int64_t npairs;       /* (J, P) pairs: J updates ancestor P                 */
  int64_t nrelind;      /* total relative-index entries                       */
  int64_t nlevels;      /* height of the supernodal elimination tree          */
  int64_t max_k, max_m; /* largest supernode width and row count              */
  double flops_alg;     /* sum_j c_j^2 over true column counts               */
  double flops_exec;    /* the same over the amalgamated (stored) structure  */
} spchol_sym_info_t;

spchol_status spchol_sym_info(spchol_sym sym, spchol_sym_info_t *info);

/* Export the structure to caller-owned host arrays (any may be NULL):
 *   parent[n]            column elimination tree of C (-1 = root)
 *   count[n]             column counts c_j of L (diagonal included)
 *   super_ptr[nsuper+1]  first column of each supernode
 *   sparent[nsuper]      supernodal elimination tree (-1 = root)
 *   row_ptr[nsuper+1], row_idx[nrows_total]   sorted row list of each supernode
 *   pair_J[npairs], pair_P[npairs]            J updates ancestor P (J ascending,
 *                                             then P ascending)
 *   pair_a0[npairs]      index, among J's off-diagonal rows, of the first row
 *                        lying in P's columns
 *   relind_ptr[npairs+1], relind[nrelind]     relind(J, P) for J's off-diagonal
 *                        rows from pair_a0 on: the distance of the row from the
 *                        bottom of P's row list, i.e. m_P - 1 - position
 *                        (Sec. II-A; positional reading of Fig. 1's example)
 *   level[nsuper]        leaves-to-root level of each supernode              */
spchol_status spchol_sym_export(spchol_sym sym, int64_t *parent, int64_t *count,
                                int64_t *super_ptr, int64_t *sparent, int64_t *row_ptr,
                                int64_t *row_idx, int64_t *pair_J, int64_t *pair_P,
                                int64_t *pair_a0, int64_t *relind_ptr, int32_t *relind,
                                int64_t *level);

/* Storage layout of the factor: supernode J is a dense column-major
 * m_J x k_J array at offset storage_off[J] (doubles) with leading dimension
 * m_J; its rows are row_idx[row_ptr[J] ...] (Sec. II-A stores each
 * supernode as a dense array).  The upper triangle of the diagonal block is
 * zero.  storage_off has nsuper+1 entries (host). */
spchol_status spchol_sym_storage(spchol_sym sym, int64_t *storage_off);

/* Numeric factorization (Sec. II-A, RL): scatter A's values into zeroed
 * supernodal storage, then per level and panel: dense Cholesky of the
 * diagonal block, triangular solve of the panel, and the update of the
 * remaining columns and of the ancestors through relative indices.
 *   vals_dev: device, fp64, colptr[n] entries in rowind's order.
 *   out: receives a new numeric handle holding L in device memory.
 *   info: host; 0 on success, else the 1-based permuted column of the
 *         smallest column whose pivot was not positive (or NaN); the status
 *         is then SPCHOL_ERR_NOT_SPD and *out is still created.
 * Synchronizes `stream` once to read the pivot status. */
spchol_status spchol_factor(spchol_sym sym, const double *vals_dev, void *stream,
                            spchol_num *out, int64_t *info);

/* Re-run the numeric factorization into an existing handle (same pattern,
 * new values), without reallocating.  Same semantics as spchol_factor; keeps
 * the update precision of the handle. */
spchol_status spchol_refactor(spchol_num num, const double *vals_dev, void *stream,
                              int64_t *info);

/* Precision of the update products (SYRK/GEMM of the panels, Sec. II-A).
 * The diagonal-block Cholesky, the triangular solves and the factor storage
 * stay fp64 in every mode; F32 (BF16) rounds the update operands to fp32
 * (bf16, round to nearest even) and accumulates in fp32 on the matrix
 * cores, then adds the result into the fp64 factor.  The factor is then that
 * of a nearby matrix: pair it with spchol_refine to recover fp64 accuracy. */
enum { SPCHOL_UPD_F64 = 0, SPCHOL_UPD_F32 = 1, SPCHOL_UPD_BF16 = 2 };

/* spchol_factor / spchol_refactor with an update precision (SPCHOL_UPD_*);
 * SPCHOL_ERR_ARG for an unsupported value. */
spchol_status spchol_factor_prec(spchol_sym sym, const double *vals_dev, int32_t update_precision,
                                 void *stream, spchol_num *out, int64_t *info);
spchol_status spchol_refactor_prec(spchol_num num, const double *vals_dev, int32_t update_precision,
                                   void *stream, int64_t *info);

/* Iterative refinement against the fp64 matrix: X = A~^{-1} B with the
 * (possibly mixed-precision) factor, then repeatedly R = B - A X (fp64,
 * original ordering), X += A~^{-1} R, until the normwise backward error
 * eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) of every column is
 * <= tol or max_iter corrections were applied.  When a correction fails to
 * halve eta of a column still above tol (refinement stalls: the reduced-
 * precision factor is too far from A for the plain iteration to contract),
 * the remaining corrections are conjugate-gradient steps on A preconditioned
 * by the factor (M = A~, symmetric positive definite), each with one solve,
 * one product with A and the same eta test.
 *   vals_dev: device, the fp64 values of A (same order as the pattern);
 *   B_dev: device, n x nrhs, leading dimension ldb (read only);
 *   X_dev: device, n x nrhs, leading dimension ldx (output);
 *   berr_out: host, nrhs entries (eta of the returned X), may be NULL;
 *   iters_out: host, corrections applied (both kinds), may be NULL;
 *   path_out: host, 0 = refinement alone, 1 = switched to preconditioned
 *             conjugate gradients, may be NULL.
 * Returns SPCHOL_ERR_NOCONV (X holds the last iterate) when the tolerance
 * is not reached.  Synchronizes `stream` once per iteration (a few times
 * per conjugate-gradient step). */
spchol_status spchol_refine(spchol_num num, const double *vals_dev, const double *B_dev,
                            double *X_dev, int64_t nrhs, int64_t ldb, int64_t ldx, double tol,
                            int32_t max_iter, void *stream, double *berr_out, int32_t *iters_out,
                            int32_t *path_out);

/* Host-resident factorization (the paper's design, Sec. III): the factor
 * lives in caller-owned host memory and the device holds only a bounded
 * working set -- the memory-capped mode for factors that do not fit the
 * device, and the host/device split by supernode size.  Supernodes with
 * k * m (columns times rows) below host_threshold are factored on the host
 * and their updates added into the ancestors there (the paper keeps them
 * on the CPU: 600,000 for its RL variant); each larger supernode is copied
 * to the device, factored by the same panel kernels, copied back, and its
 * update matrix L_RJ L_RJ^T is computed on the device in column blocks that
 * fit device_budget, each copied back and added into the ancestors by the
 * host through the relative indices (the update-block streaming of the
 * second GPU-RLB version).  host_threshold = 0 puts every supernode on the
 * device; a threshold above every k * m makes no device call at all. */
typedef struct {
  int64_t device_budget;  /* bytes for the supernode, its inverted blocks and
                             one update block (0 = 256 MiB); SPCHOL_ERR_OOM
                             when the largest device supernode plus a
                             64-column update block does not fit             */
  int64_t host_threshold; /* k * m below this: host (0 = none on the host)  */
  int32_t host_threads;   /* threads of the host parts (0 = hardware count)  */
  int32_t reserved;
} spchol_stream_options;

typedef struct {
  int64_t gpu_supernodes, host_supernodes;
  int64_t update_blocks;  /* update column blocks copied back               */
  int64_t h2d_bytes, d2h_bytes;
  int64_t device_bytes;   /* device memory the call allocated (besides the
                             analysis' device copy)                         */
  int32_t host_threads;
  int32_t reserved;
} spchol_stream_stats;

/* vals_host: host, fp64 values in the pattern's entry order; L_host: host,
 * storage doubles (layout of spchol_sym_storage; pinned memory makes the
 * copies faster), overwritten with the factor; info as spchol_factor;
 * stats: host, may be NULL.  Synchronizes `stream` (the host work needs the
 * device results).  No spchol_num is created: the factor is L_host. */
spchol_status spchol_factor_streamed(spchol_sym sym, const double *vals_host, const spchol_stream_options *opt,
                                     void *stream, double *L_host, int64_t *info, spchol_stream_stats *stats);

/* Solve A X = B in place.  B_dev: device, n x nrhs column-major, leading
 * dimension ldb >= n, original (unpermuted) ordering.  Forward solve with L
 * leaves to root, backward solve with L^T root to leaves (Sec. II).  With
 * more than four right-hand sides, groups of four alternate between
 * `stream` and the handle's second stream, which waits for `stream` first
 * and is joined back into it before the call's last launch: the call stays
 * ordered on `stream` and can be captured into a graph on it.  Asynchronous
 * (no host synchronization). */
spchol_status spchol_solve(spchol_num num, double *B_dev, int64_t nrhs, int64_t ldb,
                           void *stream);

/* spchol_solve for callers that cannot allocate device memory (code under
 * hipGraph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels and launch sequence, with the solve's work vectors in a
 * static array of this library in device memory (3 x 2^21 doubles = 48 MiB
 * per GPU, held by every GPU the call runs on until the process ends)
 * instead of buffers of the handle.  Allocates nothing (no hipMalloc,
 * hipFree, graph instantiation or event creation; per-launch profiling is
 * off for the call) and enqueues every launch eagerly on `stream`, so it
 * can itself be captured.  Requires n * nrhs <= 2^21 (SPCHOL_ERR_ARG
 * otherwise, before any device work), the current device to be the one the
 * factor lives on, and the handle's factor to exist.  Every call on one GPU
 * shares that GPU's array: calls whose work overlaps on one GPU (two
 * streams, two host threads, two handles) race and must be ordered by the
 * caller.  Each call clears the part of the array that must start at zero.
 * Arguments and result as spchol_solve. */
spchol_status spchol_solve_noalloc(spchol_num num, double *B_dev, int64_t nrhs, int64_t ldb,
                                   void *stream);

/* Reverse mode of (logdet(A), X = A^{-1} B) with respect to the stored
 * lower values of A (each off-diagonal entry stands for a_ij and a_ji) and
 * to B, for cotangents gbar_logdet (scalar) and Xbar:
 *   lam = A^{-1} Xbar,  Bbar = lam,
 *   Abar_ij = gbar w_ij Z_ij - sum_c (lam_ic x_jc + lam_jc x_ic)  (i != j),
 *   Abar_ii = gbar Z_ii - sum_c lam_ic x_ic,
 * w_ij = 2 off the diagonal, with Z = A^{-1} on the pattern obtained by
 * supernodal selected inversion (from Z L = L^{-T}; panels root to leaves).
 *   X_dev, Xbar_dev: device, n x nrhs, leading dimension ld (original
 *     ordering); Xbar_dev may be NULL (then nrhs terms are skipped);
 *   Abar_dev: device, colptr[n] entries, overwritten;
 *   Bbar_dev: device, n x nrhs with ld, may be NULL.
 * gbar_logdet = 0 skips the selected inversion. */
spchol_status spchol_backward(spchol_num num, const double *X_dev, const double *Xbar_dev,
                              int64_t nrhs, int64_t ld, double gbar_logdet, double *Abar_dev,
                              double *Bbar_dev, void *stream);

/* Normwise backward error of given solutions (Rigal-Gaches, infinity norm):
 * berr_out[c] = ||b_c - A x_c|| / (||A|| ||x_c|| + ||b_c||), the residual in
 * fp64 with the original A (values vals_dev in the pattern's entry order).
 * B_dev, X_dev: n x nrhs column-major device blocks (leading dimensions ldb,
 * ldx >= n); berr_out: host array of nrhs.  Synchronizes `stream`. */
spchol_status spchol_berr(spchol_num num, const double *vals_dev, const double *B_dev, const double *X_dev,
                          int64_t nrhs, int64_t ldb, int64_t ldx, void *stream, double *berr_out);

/* Selected inverse Z = C^{-1} (C = P A P^T) on the supernodal pattern,
 * written to caller-owned device memory in the layout of the factor
 * (spchol_sym_storage); the upper triangles of the diagonal blocks are zero,
 * as in the factor. */
spchol_status spchol_selinv_export(spchol_num num, double *dst_dev, void *stream);

/* log det(A) = 2 sum_j log L_jj, reduced on the device (pairwise tree);
 * out_host receives the value.  Synchronizes `stream`. */
spchol_status spchol_logdet(spchol_num num, double *out_host, void *stream);

/* log det of every matrix of a batch (one for a single matrix), written to
 * device memory out_dev[count]; asynchronous on `stream`. */
spchol_status spchol_logdet_batch(spchol_num num, double *out_dev, void *stream);

/* Pivot status of the last factorization enqueued into `num` (the same
 * info as spchol_factor's); synchronizes `stream`.  Needed after a graph
 * replay, which does not read it back. */
spchol_status spchol_info(spchol_num num, int64_t *info, void *stream);

/* Capture the whole numeric factorization of `num` (values from vals_dev;
 * vals_dev = NULL: no factorization, the graph only solves with the current
 * factor) and, when nrhs > 0, the solve of B_dev in place, as one hipGraph
 * on the (non-null) stream; spchol_graph_launch replays it as a single
 * launch.  The pointers are fixed in the graph: update the contents of
 * vals_dev and B_dev between replays.  The graph contains no host
 * synchronization and no memset nodes (buffers are cleared by kernels); read
 * the pivot status with spchol_info.  SPCHOL_ERR_ARG if there is nothing to
 * capture (no values and nrhs = 0).  Destroy the graph before `num`. */
spchol_status spchol_graph_create(spchol_num num, const double *vals_dev, double *B_dev, int64_t nrhs,
                                  int64_t ldb, void *stream, spchol_graph *out);
spchol_status spchol_graph_launch(spchol_graph graph, void *stream);
void spchol_graph_destroy(spchol_graph graph);

/* Copy the supernodal storage of L (storage doubles, layout as in
 * spchol_sym_storage) to caller-owned device memory dst_dev. */
spchol_status spchol_num_export(spchol_num num, double *dst_dev, void *stream);

/* Per-kernel timing of a numeric handle (HIP events recorded around every
 * launch on the call's stream while enabled).  Kernel kinds: */
enum {
  SPCHOL_KERNEL_FILL = 0,        /* zero fill of the factor storage          */
  SPCHOL_KERNEL_SCATTER_A = 1,   /* A's values into storage                  */
  SPCHOL_KERNEL_FACTOR = 2,      /* panel Cholesky + triangular solve        */
  SPCHOL_KERNEL_UPDATE_INT = 3,  /* update of a supernode's own columns      */
  SPCHOL_KERNEL_UPDATE_EXT = 4,  /* update scattered into ancestors          */
  SPCHOL_KERNEL_FWD = 5,         /* forward solve rounds                     */
  SPCHOL_KERNEL_BWD = 6,         /* backward solve rounds                    */
  SPCHOL_KERNEL_PERM = 7,        /* solve permutation gather/scatter         */
  SPCHOL_KERNEL_LOGDET = 8,
  SPCHOL_KERNEL_SELINV = 9,      /* selected inversion (reverse mode)       */
  SPCHOL_KERNEL_KINDS = 10
};

typedef struct {
  int64_t launches; /* launches timed                                          */
  double ms;        /* summed event time                                       */
  double flops;     /* algorithmic flops of those launches (stored structure)  */
  double bytes;     /* algorithmic HBM bytes of those launches                 */
} spchol_kernel_stat;

/* One timed launch.  level: the launch's level in the leaves-to-root
 * schedule of the supernodal elimination tree (Fig. 1; -1 for launches
 * outside it: fills, permutations, log-determinant, selected inversion);
 * side: 1 for external updates that ran on the second stream beside the
 * level's near updates and the next level's panel chain, else 0 (always 0
 * when every launch runs alone, profiling mode 2). */
typedef struct {
  int32_t kind;     /* SPCHOL_KERNEL_*                                         */
  int32_t level;
  int32_t side;
  int32_t reserved; /* 0                                                       */
  double ms;        /* event time of the launch                                */
  double flops;     /* algorithmic flops (stored structure)                    */
  double bytes;     /* algorithmic HBM bytes                                   */
} spchol_launch_record;

/* enable 1 or 2 starts collecting (clearing earlier records), 0 stops.
 * 1: the launches run as they do unprofiled, the external updates of a level
 * on the second stream beside other work, so their records include time
 * shared with it.  2: every launch runs alone, all on the caller's stream in
 * plan order, so each record is that launch's own duration (the factorization
 * as a whole takes longer).  SPCHOL_ERR_ARG for a null handle or another
 * value of enable. */
spchol_status spchol_profile(spchol_num num, int32_t enable);

/* Synchronize the streams the records were made on, sum the records per
 * kind into out[SPCHOL_KERNEL_KINDS] (host) and clear them. */
spchol_status spchol_profile_read(spchol_num num, spchol_kernel_stat *out);

/* The records one by one, in launch order.  *count receives the number of
 * records.  With out == NULL nothing else happens (the records are kept);
 * otherwise the first min(cap, *count) records are written to out (host
 * array, caller-owned), the streams they were made on are synchronized and
 * all records are cleared.  SPCHOL_ERR_ARG for a null handle or count, or
 * cap < 0. */
spchol_status spchol_profile_launches(spchol_num num, spchol_launch_record *out, int64_t cap, int64_t *count);

void spchol_sym_destroy(spchol_sym sym);
void spchol_num_destroy(spchol_num num);

/* Thread-local message for the last failing call on this thread. */
const char *spchol_last_error(void);

/* Library version string. */
const char *spchol_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPCHOL_H */
