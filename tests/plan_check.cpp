// Host checker of the launch schedules built by the symbolic analysis.
//
// Reads a pattern (text: n nnz, colptr, rowind, perm) and the options from
// the command line, runs the analysis and replays the factorization, forward
// and backward plans at the granularity of single entries:
//   * every entry of L receives exactly the update contributions the
//     right-looking method defines (one per earlier panel of its own
//     supernode, one per pair of off-diagonal rows of each descendant whose
//     target it is, Sec. II-A), counted independently by brute force;
//   * an entry is read by a panel factorization / triangular solve only
//     once all its contributions are in, and an update reads only solved
//     columns;
//   * inside one launch no entry is written by two tasks (unless both are
//     atomic adds) or written by one task and read by another;
//   * the solves read each panel's right-hand side only when complete and
//     never race on x.
// Prints "ok" and exits 0, or prints the first violation and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../paper_2409_14009_amd/csrc/analyze.hpp"

using namespace spchol;

namespace {

struct Access {
  // per entry: launch and task of the last writer / reader seen
  std::vector<int64_t> wl, rl;
  std::vector<int32_t> wt, rt;
  std::vector<char> wa;
  explicit Access(int64_t n) : wl(n, -1), rl(n, -1), wt(n, -1), rt(n, -1), wa(n, 0) {}
};

int64_t g_launch = 0;
std::string g_err;
// per entry: side launches forked and not yet replayed that add into it
std::vector<int32_t> g_pend;
bool g_det = false;  // deterministic schedule: not even two atomic adds per entry and launch

bool fail(const std::string& m) {
  if (g_err.empty()) g_err = m;
  return false;
}

bool on_read(Access& A, int64_t e, int32_t task) {
  if (A.wl[e] == g_launch && A.wt[e] != task) return fail("read of an entry another task of the launch writes");
  if (A.rl[e] == g_launch && A.rt[e] != task) A.rt[e] = -2;
  else if (A.rl[e] != g_launch) { A.rl[e] = g_launch; A.rt[e] = task; }
  return true;
}

bool on_write(Access& A, int64_t e, int32_t task, bool atomic) {
  if (!atomic && g_pend[e] > 0) return fail("a write of an entry a launch on another stream adds into");
  if (A.rl[e] == g_launch && A.rt[e] != task) return fail("write of an entry another task of the launch reads");
  if (A.wl[e] == g_launch && A.wt[e] != task && !(atomic && A.wa[e] && !g_det))
    return fail(g_det ? "two adds into one entry in one launch of a deterministic schedule" : "two writers in one launch");
  A.wl[e] = g_launch; A.wt[e] = task; A.wa[e] = atomic;
  return true;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 5) {
    std::fprintf(stderr, "usage: plan_check pattern.txt snode_mode amalg_z panel_width [deterministic [amalg_rule [rlb [pr]]]]\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  long long n, nz;
  if (std::fscanf(f, "%lld %lld", &n, &nz) != 2) return 2;
  std::vector<int64_t> cp(n + 1), ri(nz), pm(n);
  for (auto& v : cp) { long long x; if (std::fscanf(f, "%lld", &x) != 1) return 2; v = x; }
  for (auto& v : ri) { long long x; if (std::fscanf(f, "%lld", &x) != 1) return 2; v = x; }
  for (auto& v : pm) { long long x; if (std::fscanf(f, "%lld", &x) != 1) return 2; v = x; }
  std::fclose(f);
  Symbolic S;
  std::string err;
  g_det = argc > 5 && std::atoi(argv[5]) != 0;
  AnalyzeOptions ao;
  ao.snode_mode = std::atoi(argv[2]);
  ao.amalg_max_zeros = std::atoi(argv[3]);
  ao.panel_width = std::atoi(argv[4]);
  ao.deterministic = g_det ? 1 : 0;
  ao.amalg_rule = argc > 6 ? std::atoi(argv[6]) : 0;
  ao.update_method = argc > 7 ? std::atoi(argv[7]) : 0;
  ao.partition_refinement = argc > 8 ? std::atoi(argv[8]) : 0;
  if (analyze(n, cp.data(), ri.data(), pm.data(), ao, S, err)) {
    std::printf("analyze failed: %s\n", err.c_str());
    return 1;
  }
  const int64_t ns = S.ns, nb = S.nb, storage = S.loff[ns];
  auto K = [&](int64_t J) { return S.sptr[J + 1] - S.sptr[J]; };
  auto M = [&](int64_t J) { return S.rptr[J + 1] - S.rptr[J]; };
  auto pos_in = [&](int64_t P, int64_t row) {
    const int32_t* b = S.rows.data() + S.rptr[P];
    const int32_t* e = S.rows.data() + S.rptr[P + 1];
    const int32_t* it = std::lower_bound(b, e, (int32_t)row);
    return (it != e && *it == row) ? (int64_t)(it - b) : (int64_t)-1;
  };
  auto idx = [&](int64_t J, int64_t c, int64_t r) { return S.loff[J] + c * M(J) + r; };
  // external target of the pair (row a, row b) of J's row list, a <= b
  auto target = [&](int64_t J, int64_t a, int64_t b) -> int64_t {
    const int64_t ga = S.rows[S.rptr[J] + a], gb = S.rows[S.rptr[J] + b];
    const int64_t P = S.snode_of[ga];
    const int64_t q = pos_in(P, gb);
    if (q < 0) return -1;
    return idx(P, ga - S.sptr[P], q);
  };

  // expected contributions per entry (brute force over the definition)
  std::vector<int32_t> expect(storage, 0), got(storage, 0);
  std::vector<char> solved(storage, 0);
  for (int64_t J = 0; J < ns; ++J) {
    const int64_t k = K(J), m = M(J);
    for (int64_t c = 0; c < k; ++c)
      for (int64_t r = c; r < m; ++r) expect[idx(J, c, r)] += (int32_t)(c / nb);
    for (int64_t a = k; a < m; ++a)
      for (int64_t b = a; b < m; ++b) {
        const int64_t e = target(J, a, b);
        if (e < 0) { std::printf("row of a descendant missing in its ancestor\n"); return 1; }
        expect[e] += 1;
      }
  }

  Access acc(storage);
  auto need_complete = [&](int64_t e, int32_t t) {
    if (got[e] != expect[e]) return fail("entry factored before all its updates arrived");
    return on_read(acc, e, t);
  };
  auto solve_entry = [&](int64_t e, int32_t t) {
    if (solved[e]) return fail("entry solved twice");
    solved[e] = 1;
    return on_write(acc, e, t, false);
  };
  auto need_solved = [&](int64_t e, int32_t t) {
    if (!solved[e]) return fail("update reads a column that is not solved yet");
    return on_read(acc, e, t);
  };

  bool ok = true;
  // a launch's leading-task count (the kernel variant that takes them) lies
  // within the launch
  for (const std::vector<Launch>* plan : {&S.factor_plan, &S.fwd_plan, &S.bwd_plan, &S.si_plan})
    for (const Launch& L : *plan)
      if (L.nfirst < 0 || L.nfirst > L.ntasks) ok = fail("a launch's leading-task count exceeds its tasks");
  // a launch marked `side` (external updates of level v) runs beside the
  // launches of level v + 1 and is joined before level v + 2: it is replayed
  // at that point, after everything it may overlap with, and between fork
  // and join no launch may write (other than by atomic adds) an entry it
  // adds into.
  // The side stream forks before the near external launch of the same level
  // when that launch directly precedes it (both read the same finished
  // panels and write disjoint ancestors): a probe entry at the fork point
  // checks that every column the side launch reads is solved by then.
  std::vector<std::pair<const Launch*, bool>> order;  // (launch, probe)
  std::vector<const Launch*> pending;
  const auto& FP = S.factor_plan;
  for (size_t i = 0; i < FP.size(); ++i) {
    const Launch& L = FP[i];
    if (L.side) {
      const bool early = i > 0 && !FP[i - 1].side && (FP[i - 1].kind == K_UPD_EXT || FP[i - 1].kind == K_UPD_RLB) &&
                         FP[i - 1].level == L.level;
      if (!early) order.push_back({&L, true});
      pending.push_back(&L);
      continue;
    }
    while (!pending.empty() && L.level >= pending.front()->level + 2) {
      order.push_back({pending.front(), false});
      pending.erase(pending.begin());
    }
    if (i + 1 < FP.size() && FP[i + 1].side && (L.kind == K_UPD_EXT || L.kind == K_UPD_RLB) &&
        FP[i + 1].level == L.level)
      order.push_back({&FP[i + 1], true});
    order.push_back({&L, false});
  }
  for (const Launch* Lp : pending) order.push_back({Lp, false});
  // every entry an external tile (or RLB block tile) of launch L adds into
  auto side_targets = [&](const Launch& L, int32_t d) {
    const int64_t msk = (int64_t(1) << 25) - 1;
    for (int32_t q = 0; q < L.ntasks; ++q) {
      const Task& t = S.tasks[L.off + q];
      const int64_t m = M(t.J);
      int64_t r0 = t.a, c0 = t.b, nr = kTile, nc = kTile;
      if (L.kind == K_UPD_RLB) {
        r0 = t.a & msk; nr = (int64_t(t.a) >> 25) + 1; c0 = t.b & msk; nc = (int64_t(t.b) >> 25) + 1;
      }
      for (int64_t c = c0; c < std::min<int64_t>(c0 + nc, m); ++c)
        for (int64_t r = std::max(r0, c); r < std::min<int64_t>(r0 + nr, m); ++r) {
          const int64_t e = target(t.J, c, r);
          if (e >= 0) g_pend[e] += d;
        }
    }
  };
  g_pend.assign(storage, 0);
  int64_t fork_probes = 0;
  for (const auto& op : order) {
    const Launch& L = *op.first;
    if (op.second) {  // fork point of a side launch: its sources are final
      ++fork_probes;
      for (int32_t q = 0; q < L.ntasks && ok; ++q) {
        const int64_t J = S.tasks[L.off + q].J, k = K(J), m = M(J);
        for (int64_t s = 0; s < k && ok; ++s)
          for (int64_t r = k; r < m && ok; ++r)
            if (!solved[idx(J, s, r)]) ok = fail("side stream forked before the panel it reads is solved");
      }
      if (!ok) break;
      side_targets(L, 1);
      continue;
    }
    if (L.side) side_targets(L, -1);
    ++g_launch;
    if (L.side && L.kind != K_UPD_EXT && L.kind != K_UPD_RLB) ok = fail("side launch that is not an external update");
    for (int32_t q = 0; q < L.ntasks && ok; ++q) {
      const Task& t = S.tasks[L.off + q];
      int32_t kind = L.kind;
      if (kind == K_FACTOR_LA) kind = q < L.nfirst ? K_FACTOR : q < L.nfirst + L.ntrsm ? K_TRSM : K_UPD_INT;
      const int64_t J = t.J, k = K(J), m = M(J);
      if (kind == K_FACTOR || kind == K_TRSM) {
        const int64_t c0 = int64_t(t.a) * nb, kp = std::min<int64_t>(nb, k - c0);
        if (kind == K_FACTOR) {
          if (t.c == 1) {  // the previous panel's update of the diagonal block
            if (t.a == 0) ok = fail("diagonal pre-update without a previous panel");
            const int64_t cp = c0 - nb;
            // the whole first 64-row tile of the panel's columns
            const int64_t rE = std::min<int64_t>(c0 + kTile, m);
            for (int64_t c = c0; c < c0 + kp && ok; ++c)
              for (int64_t r = c; r < rE && ok; ++r) {
                for (int64_t s2 = cp; s2 < c0 && ok; ++s2) ok = need_solved(idx(J, s2, r), q) && need_solved(idx(J, s2, c), q);
                if (r >= c0 + kp) ok = ok && on_write(acc, idx(J, c, r), q, false);
                got[idx(J, c, r)] += 1;
              }
          } else if (t.c == 3 || t.c == 4) {
            // one-launch rounds: the block's rows in panel p-1's columns are
            // solved here (after panel p-2's update of them, c = 4), then
            // panels p-2 (c = 4) and p-1 update the diagonal block
            if (t.a < (t.c == 3 ? 1 : 2)) ok = fail("fused diagonal task without its previous panels");
            if (kp > nb || c0 - nb < 0) ok = fail("fused diagonal task outside the supernode");
            const int64_t c1 = c0 - nb, c2 = c0 - 2 * nb;
            for (int64_t s1 = c1; s1 < c0 && ok; ++s1)
              for (int64_t r = c0; r < c0 + kp && ok; ++r) {
                const int64_t e = idx(J, s1, r);
                if (t.c == 4) {
                  for (int64_t s2 = c2; s2 < c1 && ok; ++s2) ok = need_solved(idx(J, s2, r), q) && need_solved(idx(J, s2, s1), q);
                  got[e] += 1;
                }
                ok = ok && need_complete(e, q) && solve_entry(e, q);
              }
            for (int64_t c = c0; c < c0 + kp && ok; ++c)
              for (int64_t r = c; r < c0 + kp && ok; ++r) {
                for (int64_t s2 = (t.c == 4 ? c2 : c1); s2 < c0 && ok; ++s2)
                  ok = need_solved(idx(J, s2, r), q) && need_solved(idx(J, s2, c), q);
                got[idx(J, c, r)] += t.c == 4 ? 2 : 1;
              }
          } else if (t.c != 0) {
            ok = fail("unexpected FACTOR task flag");
          }
          for (int64_t c = c0; c < c0 + kp && ok; ++c)
            for (int64_t r = c; r < c0 + kp && ok; ++r) ok = need_complete(idx(J, c, r), q) && solve_entry(idx(J, c, r), q);
          const int64_t re = std::min<int64_t>(int64_t(t.b) + kTrsmRows, m);
          for (int64_t c = c0; c < c0 + kp && ok; ++c)
            for (int64_t r = t.b; r < re && ok; ++r) ok = need_complete(idx(J, c, r), q) && solve_entry(idx(J, c, r), q);
        } else {
          for (int64_t c = c0; c < c0 + kp && ok; ++c)
            for (int64_t r = c; r < c0 + kp && ok; ++r) ok = need_solved(idx(J, c, r), q);
          const int64_t re = std::min<int64_t>(int64_t(t.b) + kTile, m);
          if (t.c == 1) {  // the previous panel's update of the tile first
            if (t.a < 1) ok = fail("fused row tile without a previous panel");
            if (t.b < c0 + kp) ok = fail("fused row tile inside the diagonal block");
            for (int64_t c = c0; c < c0 + kp && ok; ++c)
              for (int64_t r = t.b; r < re && ok; ++r) {
                for (int64_t s1 = c0 - nb; s1 < c0 && ok; ++s1)
                  ok = need_solved(idx(J, s1, r), q) && need_solved(idx(J, s1, c), q);
                got[idx(J, c, r)] += 1;
              }
          } else if (t.c != 0) {
            ok = fail("unexpected TRSM task flag");
          }
          for (int64_t c = c0; c < c0 + kp && ok; ++c)
            for (int64_t r = t.b; r < re && ok; ++r) ok = need_complete(idx(J, c, r), q) && solve_entry(idx(J, c, r), q);
        }
      } else if (kind == K_SMALL) {
        // the whole supernode: every entry complete, then solved, then every
        // pair of rows below scattered (atomic adds) into its ancestors
        if (!small_supernode(k, m)) ok = fail("one-wavefront task for a supernode that does not fit");
        if (k > nb) ok = fail("one-wavefront task for a supernode wider than a panel");
        for (int64_t c = 0; c < k && ok; ++c)
          for (int64_t r = c; r < m && ok; ++r) ok = need_complete(idx(J, c, r), q) && solve_entry(idx(J, c, r), q);
        for (int64_t c = k; c < m && ok; ++c)
          for (int64_t r = c; r < m && ok; ++r) {
            const int64_t e = target(J, c, r);
            ok = on_write(acc, e, q, true);
            if (ok && solved[e]) ok = fail("update of an entry that is already solved");
            got[e] += 1;
          }
      } else if (kind == K_MEDIUM) {
        // factor and panel solve of the whole one-panel supernode (its
        // update comes from external update tiles)
        if (!medium_supernode(k, m, nb)) ok = fail("one-wavefront factor task for a supernode that does not qualify");
        if ((q < L.nfirst) != (k <= 16)) ok = fail("one-wavefront factor tasks not listed 16-column ones first");
        for (int64_t c = 0; c < k && ok; ++c)
          for (int64_t r = c; r < m && ok; ++r) ok = need_complete(idx(J, c, r), q) && solve_entry(idx(J, c, r), q);
      } else if (kind == K_UPD_INT || kind == K_UPD_EXT) {
        const bool ext = kind == K_UPD_EXT;
        // a tile over a range of panels (their adds atomic), or one panel
        const bool range = !ext && (t.c & kPanelRange);
        if (range && L.kind != K_FACTOR_LA) ok = fail("panel-range tile outside the one-launch panel rounds");
        const int64_t np = range ? ((t.c >> 16) & 0xff) : 1;
        const int64_t kb = ext ? 0 : int64_t(range ? (t.c & 0xffff) : t.c) * nb,
                      ke = ext ? k : std::min<int64_t>(k, kb + np * nb);
        const int64_t colEnd = ext ? m : k;
        if (ext && t.b < k) ok = fail("external tile that starts inside the supernode's columns");
        const int64_t r1 = std::min<int64_t>(int64_t(t.a) + kTile, m), c1 = std::min<int64_t>(int64_t(t.b) + kTile, colEnd);
        for (int64_t c = t.b; c < c1 && ok; ++c)
          for (int64_t r = std::max<int64_t>(t.a, c); r < r1 && ok; ++r) {
            for (int64_t s = kb; s < ke && ok; ++s) ok = need_solved(idx(J, s, r), q) && need_solved(idx(J, s, c), q);
            if (!ok) break;
            const int64_t e = ext ? target(J, c, r) : idx(J, c, r);
            ok = on_write(acc, e, q, ext || range);
            if (ok && solved[e]) ok = fail("update of an entry that is already solved");
            got[e] += ext ? 1 : (int32_t)((ke - kb + nb - 1) / nb);
          }
      } else if (kind == K_UPD_RLB) {
        // one block pair tile: rows and columns consecutive indices of J,
        // its columns inside one ancestor P; every entry's address from the
        // block's one relative index must be the entry's target by definition
        const int64_t msk = (int64_t(1) << 25) - 1;
        const int64_t r0 = t.a & msk, nr = (int64_t(t.a) >> 25) + 1, c0 = t.b & msk, nc = (int64_t(t.b) >> 25) + 1;
        if (c0 < k || r0 + nr > m || c0 + nc > m || r0 < c0) { ok = fail("RLB tile outside the supernode's rows"); break; }
        const int32_t* R = S.rows.data() + S.rptr[J];
        const int64_t P = S.snode_of[R[c0]];
        const int64_t mP = S.rptr[P + 1] - S.rptr[P];
        for (int64_t c = c0 + 1; c < c0 + nc && ok; ++c)
          if (R[c] != R[c - 1] + 1 || S.snode_of[R[c]] != P) ok = fail("RLB column block not consecutive in one supernode");
        for (int64_t r = r0 + 1; r < r0 + nr && ok; ++r)
          if (R[r] != R[r - 1] + 1) ok = fail("RLB row block not consecutive");
        for (int64_t c = c0; c < c0 + nc && ok; ++c)
          for (int64_t r = std::max(r0, c); r < r0 + nr && ok; ++r) {
            for (int64_t s = 0; s < k && ok; ++s) ok = need_solved(idx(J, s, r), q) && need_solved(idx(J, s, c), q);
            if (!ok) break;
            const int64_t e = target(J, c, r);
            const int64_t eb = S.loff[P] + (int64_t(R[c]) - S.sptr[P]) * mP + t.c + (r - r0);
            if (e != eb) { ok = fail("RLB block address differs from the entry's target"); break; }
            ok = on_write(acc, e, q, true);
            if (ok && solved[e]) ok = fail("update of an entry that is already solved");
            got[e] += 1;
          }
      } else {
        ok = fail("unknown launch kind in the factorization plan");
      }
    }
    if (!ok) break;
  }
  if (ok)
    for (int64_t e = 0; e < storage && ok; ++e)
      if (got[e] != expect[e]) ok = fail("an entry did not receive all its updates");
  for (int64_t J = 0; J < ns && ok; ++J)
    for (int64_t c = 0; c < K(J) && ok; ++c)
      for (int64_t r = c; r < M(J) && ok; ++r)
        if (!solved[idx(J, c, r)]) ok = fail("an entry of L was never solved");

  // forward: y[row] receives one contribution per panel whose rows below
  // contain it; a panel reads its own rows of y only when complete
  if (ok) {
    const int64_t N = S.n;
    std::vector<int32_t> ye(N, 0), yg(N, 0);
    std::vector<char> xdone(N, 0);
    for (int64_t J = 0; J < ns; ++J)
      for (int64_t p = 0; p * nb < K(J); ++p) {
        const int64_t below = p * nb + std::min<int64_t>(nb, K(J) - p * nb);
        for (int64_t r = below; r < M(J); ++r) ye[S.rows[S.rptr[J] + r]] += 1;
      }
    // a two-panel task (FWD2, c bit 1) reads panel p + 1's right-hand side
    // lacking exactly panel p's contribution, which it applies itself (the
    // first task credits it once); its tile rows get both panels'
    std::vector<int64_t> credited(N, -1);
    Access ya(N), xa(N);
    for (const Launch& L : S.fwd_plan) {
      ++g_launch;
      if (L.kind != K_FWD && L.kind != K_FWD2 && L.kind != K_FWD_SMALL) {
        ok = fail("unknown launch kind in the forward plan");
        break;
      }
      for (int32_t q = 0; q < L.ntasks && ok; ++q) {
        const Task& t = S.tasks[L.off + q];
        if (L.kind == K_FWD_SMALL) {
          // the whole supernode: z over its one panel, all rows below
          if (!small_solve_supernode(K(t.J), M(t.J), nb) || t.a != 0 || t.b != K(t.J) || t.c != 1)
            ok = fail("small forward task for a supernode that does not qualify");
          if ((q < L.nfirst) != (M(t.J) - K(t.J) <= kTile)) ok = fail("small forward tasks not listed short ones first");
          const int64_t f0 = S.sptr[t.J];
          for (int64_t i = 0; i < K(t.J) && ok; ++i) {
            if (yg[f0 + i] != ye[f0 + i]) ok = fail("forward solve reads an incomplete right-hand side");
            else ok = on_read(ya, f0 + i, q);
            if (ok && xdone[f0 + i]) ok = fail("forward solution written twice");
            xdone[f0 + i] = 1;
            ok = ok && on_write(xa, f0 + i, q, false);
          }
          for (int64_t r = K(t.J); r < M(t.J) && ok; ++r) {
            const int64_t g = S.rows[S.rptr[t.J] + r];
            ok = on_write(ya, g, q, true);
            yg[g] += 1;
          }
          continue;
        }
        const bool first = (t.c & 1) != 0, dbl = L.kind == K_FWD2 && (t.c & 2) != 0;
        if (L.kind == K_FWD && t.c != 0 && t.c != 1) ok = fail("unexpected forward task flag");
        const int64_t J = t.J, c0 = int64_t(t.a) * nb, kp = std::min<int64_t>(nb, K(J) - c0);
        const int64_t f0 = S.sptr[J] + c0;
        if (dbl && c0 + kp >= K(J)) ok = fail("two-panel task for a supernode's last panel");
        const int64_t kp1 = dbl ? std::min<int64_t>(nb, K(J) - c0 - kp) : 0, f1 = f0 + kp;
        for (int64_t i = 0; i < kp && ok; ++i) {
          if (yg[f0 + i] != ye[f0 + i]) ok = fail("forward solve reads an incomplete right-hand side");
          else ok = on_read(ya, f0 + i, q);
          if (ok && first) {
            if (xdone[f0 + i]) ok = fail("forward solution written twice");
            xdone[f0 + i] = 1;
            ok = ok && on_write(xa, f0 + i, q, false);
          }
        }
        for (int64_t i = 0; i < kp1 && ok; ++i) {
          const bool done_here = credited[f1 + i] == g_launch;
          if (yg[f1 + i] != ye[f1 + i] - (done_here ? 0 : 1))
            ok = fail("two-panel task reads an incomplete right-hand side of the second panel");
          else ok = on_read(ya, f1 + i, q);
          if (ok && first) {
            if (xdone[f1 + i]) ok = fail("forward solution written twice");
            xdone[f1 + i] = 1;
            ok = on_write(xa, f1 + i, q, false);
            if (!done_here) { yg[f1 + i] += 1; credited[f1 + i] = g_launch; }
          }
        }
        if (ok && dbl && t.b >= 0 && t.b < c0 + kp + kp1) ok = fail("two-panel tile overlaps the second panel");
        if (t.b >= 0)
          for (int64_t r = t.b; r < std::min<int64_t>(int64_t(t.b) + kTile, M(J)) && ok; ++r) {
            const int64_t g = S.rows[S.rptr[J] + r];
            ok = on_write(ya, g, q, r >= K(J));
            yg[g] += dbl ? 2 : 1;
          }
      }
      if (!ok) break;
    }
    for (int64_t i = 0; i < N && ok; ++i)
      if (!xdone[i] || yg[i] != ye[i]) ok = fail("forward solve incomplete");
    // backward: a panel is done by its single task (c = -1) or, when split,
    // by 64-row tiles (c = 0) summed into its accumulator and a finishing
    // task (c = 1 + n, n rows of its own) in a later launch; every row below
    // the panel is gathered exactly once; tasks read x below the panel,
    // which must be done, and not in the same launch
    std::vector<char> bdone(N, 0);
    std::vector<int64_t> fin_launch(N, -1), tile_launch(N, -1);
    std::vector<std::vector<char>> gathered(N);
    for (const Launch& L : S.bwd_plan) {
      ++g_launch;
      if (L.kind != K_BWD && L.kind != K_BWD_SMALL) { ok = fail("unknown launch kind in the backward plan"); break; }
      for (int32_t q = 0; q < L.ntasks && ok; ++q) {
        const Task& t = S.tasks[L.off + q];
        const int64_t J = t.J, c0 = int64_t(t.a) * nb, kp = std::min<int64_t>(nb, K(J) - c0);
        const int64_t f0 = S.sptr[J] + c0, below = c0 + kp;
        std::vector<char>& seen = gathered[f0];
        if (seen.empty()) seen.assign(M(J) - below + 1, 0);
        auto finish = [&]() {
          for (int64_t i = 0; i < kp && ok; ++i) {
            if (bdone[f0 + i]) ok = fail("backward solution written twice");
            bdone[f0 + i] = 1;
            fin_launch[f0 + i] = g_launch;
          }
        };
        auto gather = [&](int64_t r0, int64_t r1) {
          if (r0 < below || r1 > M(J)) { ok = fail("backward task rows outside the rows below its panel"); return; }
          if (bdone[f0]) { ok = fail("rows gathered for a panel already finished"); return; }
          for (int64_t r = r0; r < r1 && ok; ++r) {
            const int64_t g = S.rows[S.rptr[J] + r];
            if (seen[r - below]) ok = fail("a row gathered twice for one panel");
            else if (!bdone[g]) ok = fail("backward solve reads a row that is not solved");
            else if (fin_launch[g] == g_launch) ok = fail("backward solve reads a row solved in the same launch");
            seen[r - below] = 1;
          }
        };
        auto all_gathered = [&]() {
          for (int64_t r = below; r < M(J) && ok; ++r)
            if (!seen[r - below]) ok = fail("panel finished before all rows below it were gathered");
        };
        if (L.kind == K_BWD_SMALL) {
          if (!small_solve_supernode(K(J), M(J), nb) || t.a != 0 || t.b != below || t.c != 1)
            ok = fail("small backward task for a supernode that does not qualify");
          if ((q < L.nfirst) != (M(J) - K(J) <= kTile)) ok = fail("small backward tasks not listed short ones first");
          gather(t.b, M(J));
          all_gathered();
          finish();
        } else if (t.c < 0) {
          if (t.b != below) ok = fail("whole-panel task does not start below the panel");
          gather(t.b, M(J));
          all_gathered();
          finish();
        } else if (t.c == 0) {
          gather(t.b, std::min<int64_t>(int64_t(t.b) + kTile, M(J)));
          tile_launch[f0] = g_launch;
        } else {
          if (t.b != below) ok = fail("finishing task does not start below the panel");
          if (tile_launch[f0] == g_launch) ok = fail("panel finished in the launch of one of its tiles");
          gather(t.b, int64_t(t.b) + t.c - 1);
          all_gathered();
          finish();
        }
      }
      if (!ok) break;
    }
    for (int64_t i = 0; i < N && ok; ++i)
      if (!bdone[i]) ok = fail("backward solve incomplete");
  }
  if (!ok) {
    std::printf("violation (launch %lld): %s\n", (long long)g_launch, g_err.c_str());
    return 1;
  }
  int64_t bsplit = 0;
  for (const Launch& L : S.bwd_plan)
    if (L.kind == K_BWD)
      for (int32_t q = 0; q < L.ntasks; ++q) bsplit += S.tasks[L.off + q].c > 0;
  int64_t nsmall = 0, nfwd2 = 0, nssolve = 0, nmedium = 0;
  for (const Launch& L : S.factor_plan) {
    if (L.kind == K_SMALL) nsmall += L.ntasks;
    if (L.kind == K_MEDIUM) nmedium += L.ntasks;
  }
  for (const Launch& L : S.fwd_plan)
    if (L.kind == K_FWD_SMALL) nssolve += L.ntasks;
  for (const Launch& L : S.fwd_plan)
    if (L.kind == K_FWD2)
      for (int32_t q = 0; q < L.ntasks; ++q) nfwd2 += (S.tasks[L.off + q].c & 2) != 0;
  // algorithmic bytes the plans charge per sweep (one right-hand side)
  double fwd_bytes = 0, bwd_bytes = 0;
  for (const Launch& L : S.fwd_plan) fwd_bytes += L.bytes;
  for (const Launch& L : S.bwd_plan) bwd_bytes += L.bytes;
  int64_t rlb_tasks = 0, fused_diag = 0, range_tiles = 0;
  for (const Launch& L : S.factor_plan) {
    if (L.kind == K_UPD_RLB) rlb_tasks += L.ntasks;
    if (L.kind == K_FACTOR_LA) {
      for (int32_t q = 0; q < L.nfirst; ++q) fused_diag += S.tasks[L.off + q].c >= 3;
      for (int32_t q = L.nfirst + L.ntrsm; q < L.ntasks; ++q) range_tiles += (S.tasks[L.off + q].c & kPanelRange) != 0;
    }
  }
  std::printf("ok launches=%zu+%zu+%zu split_bwd=%lld fwd2=%lld small=%lld small_solve=%lld fwd_bytes=%.0f "
              "bwd_bytes=%.0f storage=%lld colors=%lld si_launches=%zu rlb_blocks=%lld rlb_tasks=%lld fused_diag=%lld fork_probes=%lld medium=%lld range_tiles=%lld\n",
              S.factor_plan.size(), S.fwd_plan.size(), S.bwd_plan.size(), (long long)bsplit, (long long)nfwd2,
              (long long)nsmall, (long long)nssolve, fwd_bytes, bwd_bytes, (long long)storage,
              (long long)S.max_colors, S.si_plan.size(), (long long)S.rlb_blocks, (long long)rlb_tasks,
              (long long)fused_diag, (long long)fork_probes, (long long)nmedium, (long long)range_tiles);
  return 0;
}
