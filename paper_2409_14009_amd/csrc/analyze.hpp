// Host-side symbolic analysis and launch-schedule construction.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "consts.hpp"

namespace spchol {

// Work item of a batched launch.  Meaning of the fields per launch kind:
//   FACTOR     J, panel, first local row the task solves itself (up to
//              kTrsmRows rows from there; == m_J: none), 1 when the task
//              first applies the previous panel's update to its diagonal
//              block (else 0)
//   FACTOR_LA  the first `nfirst` tasks are FACTOR tasks, the others
//              UPD_INT tiles of the previous panel that do not touch the
//              panel being factored (one-panel lookahead)
//   TRSM       J, panel, first local row of a further 64-row tile, -
//   UPD_INT    J, first local row (target rows), first local col (target
//              cols), panel (the K range)
//   UPD_EXT    J, first local row, first local col, -1
//   UPD_RLB    J, first local row | (rows - 1) << 25, first local col |
//              (cols - 1) << 25, position of the first row in the target
//              supernode's row list: a tile of one block pair (Sec. II-B),
//              its rows consecutive in J and in the target, its columns
//              consecutive in the target's columns
//   SMALL      J, -, -, -  (factor, inverse block and external update of
//              a supernode for which small_supernode holds)
//   FWD        J, panel, first local row of a 64-row tile below the panel
//              (-1: the panel has no rows below), 1 on the panel's first task
//   FWD2       as FWD; c bit 1 set: the task covers panels p and p + 1 (its
//              tile lies below panel p + 1; bit 0: it also stores both
//              panels' solution)
//   FWD_SMALL, BWD_SMALL  J, 0, k_J, 1 (a supernode for which
//              small_solve_supernode holds: all its rows in one task)
//   BWD        J, panel, first local row of the task's rows, and -1 (all
//              rows below the panel, then the diagonal block), 0 (one 64-row
//              tile, summed into the accumulator) or 1 + n (n rows, then the
//              accumulator and the diagonal block)
struct Task {
  int32_t J, a, b, c;
};

enum Kind : int32_t {
  K_FACTOR = 0,
  K_UPD_INT = 1,
  K_UPD_EXT = 2,
  K_FWD = 3,    // forward solve round: inverse-block product + panel update
  K_BWD = 4,    // backward solve round: panel gathers, inverse-block products
  K_TRSM = 7,
  K_SI_W = 8,   // (unused: the factorization stores the inverted diagonal blocks)
  K_SI_Y = 9,   // Y = Z_BB L_Bp tiles
  K_SI_ZB = 10, // Z_Bp = -Y W tiles (+ T)
  K_SI_ZD = 11, // Z_pp = (W^T - T) W
  K_FACTOR_LA = 12,
  K_SMALL = 13,  // a supernode whose whole numeric step fits one wavefront
  K_FWD2 = 14,   // forward solve round with two-panel tasks
  K_FWD_SMALL = 15,  // forward solve of small one-panel supernodes, one wavefront each
  K_BWD_SMALL = 16,  // backward solve of the same
  K_UPD_RLB = 17,    // external update by block pairs (RLB)
  K_MEDIUM = 18,     // a short one-panel supernode of at most 32 columns not done by K_SMALL:
                     // factor, inverse block and all rows below in one wavefront
};

// Supernodes done by one wavefront (K_SMALL): at most 16 columns, and with
// the swept block padded to 4 (K <= 4) or 16 columns, the padded block, the
// rows below and one unit row per column (for the inverse block) fit the
// wavefront's 64 lanes.
inline bool small_supernode(int64_t k, int64_t m) { return k <= 16 && (k <= 4 ? 4 : 16) + m <= 64; }

// Supernodes factored by one wavefront without their update (K_MEDIUM): at
// most 32 columns (one panel), at most kMediumRows rows below, not done by
// K_SMALL; the diagonal block, the inverse block and every row below are
// done by the wavefront (the rows past its sweep 64 at a time, in
// sequence: taller panels go to the row tiles, which run in parallel), the
// update goes to the external update tiles.  A K_MEDIUM launch lists its
// supernodes of at most 16 columns first (nfirst of them).
constexpr int64_t kMediumRows = 160;
constexpr int64_t kMediumMin = 128;  // fewer in a level that also has panel rounds: they join those
inline bool medium_supernode(int64_t k, int64_t m, int64_t nb) {
  return k <= 32 && k <= nb && m - k <= kMediumRows && !small_supernode(k, m);
}

// Supernodes solved by one wavefront (K_FWD_SMALL, K_BWD_SMALL): one panel
// of at most 16 columns and at most 128 rows below it (two per lane).  A
// level gets such a launch when it holds at least kSmallSolveMin of them
// (else they stay in the level's ordinary rounds: one launch fewer).
inline bool small_solve_supernode(int64_t k, int64_t m, int64_t nb) { return k <= 16 && k <= nb && m - k <= 128; }
constexpr int64_t kSmallSolveMin = 256;

struct Launch {
  int32_t kind;
  int32_t ntasks;
  int64_t off;  // first task in the task array
  int32_t level;
  int32_t panel;
  double flops = 0;  // algorithmic flops of the launch (stored structure)
  double bytes = 0;  // algorithmic HBM bytes of the launch
  int64_t slot_base = 0;  // selected inversion: first entry of si_yoff for this round
  int32_t seg = 0;        // SI_Y: rows of B per task (64, 128 or kSiSeg)
  int32_t nfirst = 0;     // FACTOR_LA: number of leading FACTOR tasks; MEDIUM: of those with at
                          // most 16 columns; FWD_SMALL / BWD_SMALL: of those with at most 64 rows below
  int32_t ntrsm = 0;      // FACTOR_LA: number of TRSM tasks after them (the one-launch
                          // panel rounds; the rest are internal update tiles)
  int32_t side = 0;       // UPD_EXT of level l whose targets lie above level l+1: may run
                          // beside level l+1's launches, must finish before level l+2's
};

constexpr int kTile = 64;      // rows (and cols) of an update tile
constexpr int kTrsmRows = 256; // rows solved by the diagonal-block workgroup
constexpr int kInlineMinTasks = 128;  // launches with fewer diagonal tasks solve no rows inline
constexpr int kBwdRows = 256;  // backward solve: taller panels are split into row tiles
constexpr int kMaxPanel = 64;  // largest panel width

struct Symbolic {
  int64_t n = 0, nnzA = 0;
  int nb = 64;  // panel width
  std::vector<int64_t> perm, pinv;
  std::vector<int64_t> parent, count;  // column etree and column counts of L
  int64_t ns = 0;
  std::vector<int64_t> sptr;     // ns+1, first column of each supernode
  std::vector<int64_t> sparent;  // ns
  std::vector<int64_t> rptr;     // ns+1, offsets of the row lists
  std::vector<int32_t> rows;     // concatenated sorted row lists
  std::vector<int64_t> loff;     // ns+1, storage offsets (doubles)
  std::vector<int64_t> obase;    // ns+1, offsets of per-off-diagonal-row arrays
  std::vector<int32_t> opair;    // pair id of each off-diagonal row
  std::vector<int64_t> ocbase;   // storage offset of the target column of each off-diagonal row
  std::vector<int64_t> pJ, pP, pa0, relptr;
  std::vector<int32_t> tpos;     // position (from the top) of the row in P's row list
  std::vector<int64_t> level;    // per supernode
  std::vector<int64_t> amap;     // nnzA: storage offset of each entry of A
  std::vector<int64_t> snode_of; // n: supernode of each column
  // full-symmetric CSR of A in the original ordering; each entry indexes the
  // stored lower-triangle value array (residuals of iterative refinement)
  std::vector<int64_t> a_rp, a_vidx;
  std::vector<int32_t> a_col;
  int64_t nlevels = 0;
  int64_t max_k = 0, max_m = 0;
  // inverted diagonal blocks of all panels (written by the factorization,
  // read by its row tiles and the solves): panel p of J at
  // wbase[J] + p * nb * nb, kp x kp column-major
  std::vector<int64_t> wbase;  // ns+1

  double flops_alg = 0, flops_exec = 0;
  // schedule
  std::vector<Task> tasks;
  std::vector<Launch> factor_plan, fwd_plan, bwd_plan, si_plan;
  std::vector<int64_t> si_yoff;  // per selected-inversion slot: offset of its Y block
  int64_t si_max_slots = 0, si_max_y = 0;
  std::vector<int32_t> e_row, e_col;  // row and column of each stored entry of A
  // deterministic schedule: no launch holds two tasks that add into one
  // entry (the adds of a level go in launches of disjoint targets, in a
  // fixed order), so every run gives the same bits
  bool deterministic = false;
  int64_t max_colors = 0;  // most launches one scatter launch was split into
  int update_method = 0;   // 0 RL, 1 RLB
  int64_t rlb_blocks = 0;  // RLB: row blocks over all supernodes updated by tiles
};

// Returns 0, or a negative spchol_status with a message in err.
// Options of the analysis (the C ABI's spchol_options).
struct AnalyzeOptions {
  int snode_mode = 0;       // 0 fundamental, 1 maximal supernodes
  int amalg_max_zeros = 0;  // amalg_rule 0: explicit zeros allowed per column
  int panel_width = 64;
  int deterministic = 0;    // schedule without two adds into one entry per launch
  int amalg_rule = 0;       // 0: per-column zero cap; 1: greedy least-new-fill merging (Sec. IV-A)
  int amalg_cap_percent = 25;  // amalg_rule 1: storage increase allowed, percent of nnz(L)
  int update_method = 0;    // 0: RL (update tiles scattered row by row through
                            // relative indices); 1: RLB (Sec. II-B: block pairs of
                            // consecutive rows, one relative index per block)
  int partition_refinement = 0;  // reorder the columns of every supernode so that the
                                 // rows of its descendants form fewer, longer blocks
};

// Returns 0, or a negative spchol_status with a message in err.
int analyze(int64_t n, const int64_t* colptr, const int64_t* rowind, const int64_t* perm, const AnalyzeOptions& o,
            Symbolic& S, std::string& err);

}  // namespace spchol
