// Fill-reducing ordering of a general sparse symmetric pattern.
#pragma once
#include <cstdint>
#include <string>

namespace spchol {

// Nested dissection by multilevel bisection (order.cpp): perm[k] = the
// original index eliminated k-th.  The pattern is a CSC lower (or full)
// triangle; rows may be in any order, duplicates are harmless.  Subgraphs of
// at most `leaf` vertices are ordered by minimum degree.  Returns 0, or a
// negative spchol_status with a message in err.
int order_nd(int64_t n, const int64_t* colptr, const int64_t* rowind, int64_t leaf, uint64_t seed, int64_t* perm,
             std::string& err);

}  // namespace spchol
