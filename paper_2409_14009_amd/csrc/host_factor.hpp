// Host-side numeric steps of the host-resident factorization.
#pragma once
#include <cstdint>

#include "analyze.hpp"

namespace spchol {

// L (host, storage doubles) <- zero, then A's values at their positions.
void host_scatter_values(const Symbolic& S, const double* vals, double* L);

// Dense Cholesky of supernode J's m x k storage in place (its updates from
// descendants already applied); returns the first failing (permuted,
// 0-based) column, or -1.
int64_t host_factor_supernode(const Symbolic& S, int64_t J, double* L);

// Subtract J's update L_RJ L_RJ^T from its ancestors through the relative
// indices (J factored).
void host_update_supernode(const Symbolic& S, int64_t J, double* L, int threads);

// Subtract columns cb .. ce - 1 (local rows of J) of J's update matrix, given
// as U (rows cb .. m_J - 1, column-major, leading dimension m_J - cb), from
// the ancestors.
void host_assemble_block(const Symbolic& S, int64_t J, int64_t cb, int64_t ce, const double* U, double* L,
                         int threads);

}  // namespace spchol
