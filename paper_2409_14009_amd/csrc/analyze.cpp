// Symbolic analysis for the right-looking supernodal Cholesky.
//
// Steps (host, linear or near-linear in the size of L's supernodal
// structure):
//   1. C = P A P^T, lower pattern, by rows and by columns.
//   2. Elimination tree (Sec. II: the parent of column j is the smallest
//      off-diagonal row of L_{*,j}) by Liu's algorithm with path compression.
//   3. Column counts of L by walking each row subtree of the etree.
//   4. Supernodes (Sec. I): column j+1 continues j's supernode when
//      parent(j) = j+1 and c_j = c_{j+1} + 1 (then struct(L_j) \ {j} equals
//      struct(L_{j+1}) by the containment of Sec. II); the fundamental mode
//      also needs j to be the only child of j+1.
//   5. Relaxed amalgamation (Sec. IV-A merges supernodes with their parents):
//      a chain of supernodes is merged into a parent that starts right after
//      it when the merged dense storage has at most z explicit zeros per
//      column.  Counted arithmetically from the column counts.
//   6. Supernodal row lists, the supernodal etree (Fig. 1) and relative
//      indices relind(J, P) (Sec. II-A): for each ancestor P holding one of
//      J's off-diagonal rows, the position of J's rows in P's row list.
//   7. Storage offsets, the map of A's entries into storage, levels and the
//      batched launch schedule.
#include "analyze.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <queue>
#include <tuple>

namespace spchol {

namespace {

constexpr int ERR_ARG = -1, ERR_PATTERN = -2, ERR_OOM = -4;

}  // namespace

int analyze(int64_t n, const int64_t* colptr, const int64_t* rowind, const int64_t* perm, const AnalyzeOptions& o,
            Symbolic& S, std::string& err) {
  const int snode_mode = o.snode_mode, amalg_max_zeros = o.amalg_max_zeros, panel_width = o.panel_width;
  const int deterministic = o.deterministic, amalg_rule = o.amalg_rule, amalg_cap_percent = o.amalg_cap_percent;
  if (o.update_method != 0 && o.update_method != 1) { err = "analyze: bad update_method"; return ERR_ARG; }
  try {
    if (n < 0 || !colptr || (n > 0 && !rowind)) { err = "analyze: null pointer or n < 0"; return ERR_ARG; }
    if (n >= (int64_t(1) << 31) - 1) { err = "analyze: n too large (rows are stored as int32)"; return ERR_ARG; }
    if (snode_mode != 0 && snode_mode != 1) { err = "analyze: bad snode_mode"; return ERR_ARG; }
    if (amalg_max_zeros < 0) { err = "analyze: amalg_max_zeros < 0"; return ERR_ARG; }
    if (amalg_rule != 0 && amalg_rule != 1) { err = "analyze: bad amalg_rule"; return ERR_ARG; }
    if (amalg_cap_percent < 0) { err = "analyze: amalg_cap_percent < 0"; return ERR_ARG; }
    int nb = panel_width == 0 ? 64 : panel_width;
    if (nb < 16 || nb > kMaxPanel || nb % 16) { err = "analyze: panel_width must be 16, 32, 48 or 64"; return ERR_ARG; }
    S = Symbolic();
    S.n = n;
    S.nb = nb;
    S.deterministic = deterministic != 0;
    S.update_method = o.update_method;
    if (colptr[0] != 0) { err = "analyze: colptr[0] != 0"; return ERR_PATTERN; }
    for (int64_t j = 0; j < n; ++j)
      if (colptr[j + 1] < colptr[j]) { err = "analyze: colptr not monotone"; return ERR_PATTERN; }
    const int64_t nz = colptr[n];
    S.nnzA = nz;
    for (int64_t j = 0; j < n; ++j) {
      if (colptr[j] == colptr[j + 1] || rowind[colptr[j]] != j) {
        err = "analyze: missing diagonal entry in column " + std::to_string(j);
        return ERR_PATTERN;
      }
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        int64_t i = rowind[p];
        if (i < j || i >= n) { err = "analyze: entry outside the lower triangle in column " + std::to_string(j); return ERR_PATTERN; }
        if (p > colptr[j] && i <= rowind[p - 1]) { err = "analyze: rows not strictly increasing in column " + std::to_string(j); return ERR_PATTERN; }
      }
    }
    // ---- permutation ------------------------------------------------------
    S.perm.resize(n);
    S.pinv.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      int64_t o = perm ? perm[k] : k;
      if (o < 0 || o >= n || S.pinv[o] != -1) { err = "analyze: perm is not a permutation"; return ERR_ARG; }
      S.perm[k] = o;
      S.pinv[o] = k;
    }
    // ---- 1. C = P A P^T lower, by rows (strict) and by columns ------------
    std::vector<int64_t> rp(n + 1, 0), cp(n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        int64_t a = S.pinv[rowind[p]], b = S.pinv[j];
        int64_t r = std::max(a, b), c = std::min(a, b);
        if (r != c) rp[r + 1]++;
        cp[c + 1]++;
      }
    for (int64_t i = 0; i < n; ++i) { rp[i + 1] += rp[i]; cp[i + 1] += cp[i]; }
    std::vector<int32_t> rc(rp[n]), cr(cp[n]);
    {
      std::vector<int64_t> fr(rp.begin(), rp.end() - 1), fc(cp.begin(), cp.end() - 1);
      for (int64_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
          int64_t a = S.pinv[rowind[p]], b = S.pinv[j];
          int64_t r = std::max(a, b), c = std::min(a, b);
          if (r != c) rc[fr[r]++] = (int32_t)c;
          cr[fc[c]++] = (int32_t)r;
        }
    }
    // ---- 2. elimination tree (Liu, path compression) ---------------------
    S.parent.assign(n, -1);
    {
      std::vector<int64_t> anc(n, -1);
      for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
          int64_t r = rc[p];
          while (anc[r] != -1 && anc[r] != i) {
            int64_t nx = anc[r];
            anc[r] = i;
            r = nx;
          }
          if (anc[r] == -1) {
            anc[r] = i;
            S.parent[r] = i;
          }
        }
      }
    }
    // ---- 3. column counts by row-subtree walks ----------------------------
    S.count.assign(n, 0);
    {
      std::vector<int64_t> mark(n, -1);
      for (int64_t i = 0; i < n; ++i) {
        S.count[i] += 1;
        mark[i] = i;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
          int64_t k = rc[p];
          while (mark[k] != i) {
            S.count[k] += 1;
            mark[k] = i;
            k = S.parent[k];
          }
        }
      }
    }
    for (int64_t j = 0; j < n; ++j) S.flops_alg += double(S.count[j]) * double(S.count[j]);
    // ---- 4. base supernodes ---------------------------------------------
    std::vector<int64_t> nchild(n, 0);
    for (int64_t j = 0; j < n; ++j)
      if (S.parent[j] >= 0) nchild[S.parent[j]]++;
    std::vector<int64_t> bptr;
    bptr.reserve(n + 1);
    for (int64_t j = 0; j < n; ++j) {
      bool cont = j > 0 && S.parent[j - 1] == j && S.count[j - 1] == S.count[j] + 1 &&
                  (snode_mode == 1 || nchild[j] == 1);
      if (!cont) bptr.push_back(j);
    }
    bptr.push_back(n);
    const int64_t nbase = (int64_t)bptr.size() - 1;
    std::vector<int64_t> bsn(n);
    for (int64_t b = 0; b < nbase; ++b)
      for (int64_t j = bptr[b]; j < bptr[b + 1]; ++j) bsn[j] = b;
    // ---- 5. amalgamation (arithmetic on counts) ---------------------------
    // A group is a run of base supernodes ending at base supernode b; its
    // rows are its columns plus the off-diagonal rows of b, so m = (columns
    // of the group) + (rows of b below b).  Merging the group into the base
    // parent p (which starts right after it) gives k = cols(group) + k_p and
    // m = cols(group) + m_p.
    std::vector<int64_t> gfirst(nbase), gtrue(nbase);
    std::vector<char> alive(nbase, 1);
    for (int64_t b = 0; b < nbase; ++b) {
      gfirst[b] = bptr[b];
      int64_t t = 0;
      for (int64_t j = bptr[b]; j < bptr[b + 1]; ++j) t += S.count[j];
      gtrue[b] = t;
    }
    if (amalg_rule == 1) {
      // Sec. IV-A: merge supernode pairs (J, p(J)) in sequence, each step
      // the pair adding the least new fill, until the cumulative increase
      // of the factor's storage would pass amalg_cap_percent of nnz(L).
      // Candidates: a group and the group holding its parent column, when
      // that group starts right after it (merged columns stay consecutive).
      // New fill of merging G (K_G, M_G) into Q (K_Q, M_Q): the merged
      // trapezoid (K_G + K_Q columns, K_G + M_Q rows) minus both trapezoids,
      // K_G (K_G + M_Q - M_G).  Ties: the group with the smaller first column.
      std::vector<int64_t> gend(nbase);  // union-find: base -> end of its group
      std::iota(gend.begin(), gend.end(), 0);
      auto find = [&](int64_t b) {
        while (gend[b] != b) { gend[b] = gend[gend[b]]; b = gend[b]; }
        return b;
      };
      auto Kg = [&](int64_t e) { return bptr[e + 1] - gfirst[e]; };
      auto Mg = [&](int64_t e) { return (bptr[e] - gfirst[e]) + S.count[bptr[e]]; };
      // the candidate of group e (its end): the group q holding its parent
      // column, if q starts right after e; -1 otherwise
      auto target = [&](int64_t e) -> int64_t {
        const int64_t pc = S.parent[bptr[e + 1] - 1];
        if (pc < 0) return -1;
        const int64_t q = find(bsn[pc]);
        return gfirst[q] == bptr[e + 1] ? q : -1;
      };
      auto cost = [&](int64_t e, int64_t q) { return Kg(e) * (Kg(e) + Mg(q) - Mg(e)); };
      std::vector<int64_t> stamp(nbase, 0);
      using Cand = std::tuple<int64_t, int64_t, int64_t, int64_t>;  // cost, first column, end, stamp
      std::priority_queue<Cand, std::vector<Cand>, std::greater<Cand>> pq;
      auto push = [&](int64_t e) {
        const int64_t q = target(e);
        if (q >= 0) pq.push(Cand{cost(e, q), gfirst[e], e, stamp[e]});
      };
      for (int64_t b = 0; b < nbase; ++b) push(b);
      int64_t nnzl = 0;
      for (int64_t j = 0; j < n; ++j) nnzl += S.count[j];
      const int64_t cap = nnzl * (int64_t)amalg_cap_percent / 100;
      int64_t added = 0;
      while (!pq.empty()) {
        const auto [c, f, e, st] = pq.top();
        pq.pop();
        if (!alive[e] || st != stamp[e]) continue;
        const int64_t q = target(e);
        if (q < 0 || cost(e, q) != c) { ++stamp[e]; push(e); continue; }
        if (added + c > cap) break;
        added += c;
        gfirst[q] = gfirst[e];
        gtrue[q] += gtrue[e];
        alive[e] = 0;
        gend[e] = q;
        // q's own candidate and that of the group ending just before it
        // (whose parent may lie in q now) change
        ++stamp[q];
        push(q);
        if (gfirst[q] > 0) {
          const int64_t prev = find(bsn[gfirst[q] - 1]);
          ++stamp[prev];
          push(prev);
        }
      }
    } else if (amalg_max_zeros > 0) {
      const int64_t z = amalg_max_zeros;
      for (int64_t b = 0; b < nbase; ++b) {
        int64_t last = bptr[b + 1] - 1;
        int64_t pc = S.parent[last];
        if (pc < 0) continue;
        int64_t p = bsn[pc];
        if (bptr[p] != last + 1) continue;
        int64_t gcols = bptr[p] - gfirst[b];
        int64_t mp = S.count[bptr[p]];  // rows of base supernode p
        int64_t k = gcols + (bptr[p + 1] - bptr[p]);
        int64_t m = gcols + mp;
        int64_t storage = k * m - k * (k - 1) / 2;
        int64_t zeros = storage - (gtrue[b] + gtrue[p]);
        if (zeros <= z * k) {
          gfirst[p] = gfirst[b];
          gtrue[p] += gtrue[b];
          alive[b] = 0;
        }
      }
    }
    // ---- 6. final supernodes, row lists ----------------------------------
    std::vector<int64_t> fin;  // base supernode that ends each final supernode
    for (int64_t b = 0; b < nbase; ++b)
      if (alive[b]) fin.push_back(b);
    const int64_t ns = (int64_t)fin.size();
    S.ns = ns;
    S.sptr.resize(ns + 1);
    for (int64_t J = 0; J < ns; ++J) S.sptr[J] = gfirst[fin[J]];
    S.sptr[ns] = n;
    S.snode_of.resize(n);
    for (int64_t J = 0; J < ns; ++J)
      for (int64_t j = S.sptr[J]; j < S.sptr[J + 1]; ++j) S.snode_of[j] = J;
    S.sparent.resize(ns);
    for (int64_t J = 0; J < ns; ++J) {
      int64_t pc = S.parent[S.sptr[J + 1] - 1];
      S.sparent[J] = pc < 0 ? -1 : S.snode_of[pc];
    }
    // Row lists of base supernodes: the columns, the entries of C below the
    // supernode, and the rows of the child supernodes below it.
    std::vector<int64_t> brp(nbase + 1, 0);
    std::vector<int32_t> brows;
    {
      std::vector<int64_t> mark(n, -1);
      std::vector<std::vector<int64_t>> kids(nbase);
      for (int64_t b = 0; b < nbase; ++b) {
        int64_t pc = S.parent[bptr[b + 1] - 1];
        if (pc >= 0) kids[bsn[pc]].push_back(b);
      }
      std::vector<int32_t> tmp;
      for (int64_t b = 0; b < nbase; ++b) {
        tmp.clear();
        int64_t f = bptr[b], l = bptr[b + 1] - 1;
        for (int64_t j = f; j <= l; ++j) { tmp.push_back((int32_t)j); mark[j] = b; }
        for (int64_t j = f; j <= l; ++j)
          for (int64_t p = cp[j]; p < cp[j + 1]; ++p) {
            int64_t i = cr[p];
            if (i > l && mark[i] != b) { mark[i] = b; tmp.push_back((int32_t)i); }
          }
        for (int64_t c : kids[b])
          for (int64_t p = brp[c]; p < brp[c + 1]; ++p) {
            int64_t i = brows[p];
            if (i > l && mark[i] != b) { mark[i] = b; tmp.push_back((int32_t)i); }
          }
        std::sort(tmp.begin() + (l - f + 1), tmp.end());
        if ((int64_t)tmp.size() != S.count[f]) { err = "analyze: internal error (row list vs column count)"; return ERR_PATTERN; }
        brows.insert(brows.end(), tmp.begin(), tmp.end());
        brp[b + 1] = (int64_t)brows.size();
      }
    }
    // final row list = the merged columns before the last base supernode,
    // then that base supernode's rows
    S.rptr.assign(ns + 1, 0);
    for (int64_t J = 0; J < ns; ++J) {
      int64_t b = fin[J];
      S.rptr[J + 1] = S.rptr[J] + (bptr[b] - S.sptr[J]) + (brp[b + 1] - brp[b]);
    }
    S.rows.resize(S.rptr[ns]);
    for (int64_t J = 0; J < ns; ++J) {
      int64_t b = fin[J], q = S.rptr[J];
      for (int64_t j = S.sptr[J]; j < bptr[b]; ++j) S.rows[q++] = (int32_t)j;
      for (int64_t p = brp[b]; p < brp[b + 1]; ++p) S.rows[q++] = brows[p];
    }
    brows.clear(); brows.shrink_to_fit();
    // storage offsets, sizes, executed flops
    S.loff.assign(ns + 1, 0);
    S.obase.assign(ns + 1, 0);
    S.wbase.assign(ns + 1, 0);
    for (int64_t J = 0; J < ns; ++J) {
      int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
      S.loff[J + 1] = S.loff[J] + k * m;
      // inverted diagonal blocks: full panels nb x nb, the last kp x kp
      S.wbase[J + 1] = S.wbase[J] + (k / S.nb) * S.nb * S.nb + (k % S.nb) * (k % S.nb);
      S.obase[J + 1] = S.obase[J] + (m - k);
      S.max_k = std::max(S.max_k, k);
      S.max_m = std::max(S.max_m, m);
      for (int64_t t = 0; t < k; ++t) S.flops_exec += double(m - t) * double(m - t);
    }
    // ---- partition refinement ----------------------------------------
    // Reorder the columns inside every supernode P so that the rows of each
    // descendant J lying in P's columns become consecutive: the columns of P
    // are ordered by refining the partition {cols(P)} with those row sets,
    // largest first, each part X splitting into X n S before X \ S (stable),
    // which makes every set of a nested or disjoint family consecutive.  The
    // supernodal structure is kept as it is, relabelled: the partition, the
    // diagonal blocks (stored dense) and the sets of rows below each
    // supernode do not depend on the order of the columns inside a
    // supernode (block elimination on the same partition), so neither does
    // the storage (Sec. IV-A: reordering within supernodes leaves the fill
    // unchanged).  The elimination order becomes perm composed with the
    // relabelling (S.perm); parent and count are the unrefined ones mapped
    // through it.
    if (o.partition_refinement) {
      std::vector<std::vector<std::pair<int64_t, int64_t>>> sets(ns);  // (start in rows, length) per target
      for (int64_t J = 0; J < ns; ++J) {
        const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
        const int32_t* R = S.rows.data() + S.rptr[J];
        for (int64_t a = k; a < m;) {
          const int64_t P = S.snode_of[R[a]];
          int64_t b = a;
          while (b < m && R[b] < S.sptr[P + 1]) ++b;
          sets[P].push_back({S.rptr[J] + a, b - a});
          a = b;
        }
      }
      std::vector<int64_t> newidx(n);
      std::vector<char> in(n, 0);
      std::vector<int64_t> cur, pid, ncur, npid;
      for (int64_t P = 0; P < ns; ++P) {
        const int64_t f = S.sptr[P], l = S.sptr[P + 1];
        auto& st = sets[P];
        std::stable_sort(st.begin(), st.end(), [](const std::pair<int64_t, int64_t>& a,
                                                  const std::pair<int64_t, int64_t>& b) { return a.second > b.second; });
        cur.resize(l - f);
        pid.assign(l - f, 0);
        for (int64_t c = f; c < l; ++c) cur[c - f] = c;
        for (const auto& e : st) {
          if (e.second == l - f) continue;  // the whole supernode: splits nothing
          for (int64_t q = e.first; q < e.first + e.second; ++q) in[S.rows[q]] = 1;
          ncur.clear();
          npid.clear();
          int64_t np = 0;
          for (size_t i = 0; i < cur.size();) {
            size_t j = i;
            while (j < cur.size() && pid[j] == pid[i]) ++j;
            for (int pass = 0; pass < 2; ++pass) {
              bool any = false;
              for (size_t q = i; q < j; ++q)
                if ((bool)in[cur[q]] == (pass == 0)) { ncur.push_back(cur[q]); npid.push_back(np); any = true; }
              if (any) ++np;
            }
            i = j;
          }
          cur.swap(ncur);
          pid.swap(npid);
          for (int64_t q = e.first; q < e.first + e.second; ++q) in[S.rows[q]] = 0;
        }
        for (int64_t i = 0; i < l - f; ++i) newidx[cur[i]] = f + i;
      }
      std::vector<int64_t> nperm(n), npar(n), ncnt(n);
      for (int64_t c = 0; c < n; ++c) {
        nperm[newidx[c]] = S.perm[c];
        npar[newidx[c]] = S.parent[c] < 0 ? -1 : newidx[S.parent[c]];
        ncnt[newidx[c]] = S.count[c];
      }
      S.perm.swap(nperm);
      S.parent.swap(npar);
      S.count.swap(ncnt);
      for (int64_t c = 0; c < n; ++c) S.pinv[S.perm[c]] = c;
      for (int64_t J = 0; J < ns; ++J) {
        const int64_t k = S.sptr[J + 1] - S.sptr[J];
        int32_t* R = S.rows.data() + S.rptr[J];
        const int64_t m = S.rptr[J + 1] - S.rptr[J];
        for (int64_t a = 0; a < m; ++a) R[a] = (int32_t)newidx[R[a]];
        std::sort(R, R + k);
        std::sort(R + k, R + m);
      }
    }
    if (S.update_method == 1 && S.max_m >= (int64_t(1) << 25)) {
      err = "analyze: a supernode has too many rows for the RLB task encoding";
      return ERR_ARG;
    }
    // ---- relative indices ---------------------------------------------
    S.opair.resize(S.obase[ns]);
    S.ocbase.resize(S.obase[ns]);
    S.relptr.push_back(0);
    for (int64_t J = 0; J < ns; ++J) {
      int64_t k = S.sptr[J + 1] - S.sptr[J];
      const int32_t* R = S.rows.data() + S.rptr[J] + k;
      int64_t r = S.rptr[J + 1] - S.rptr[J] - k;
      int64_t a = 0;
      while (a < r) {
        int64_t P = S.snode_of[R[a]];
        int64_t pid = (int64_t)S.pJ.size();
        S.pJ.push_back(J);
        S.pP.push_back(P);
        S.pa0.push_back(a);
        const int32_t* PR = S.rows.data() + S.rptr[P];
        int64_t mP = S.rptr[P + 1] - S.rptr[P], q = 0;
        for (int64_t c = a; c < r; ++c) {
          while (q < mP && PR[q] < R[c]) ++q;
          if (q >= mP || PR[q] != R[c]) { err = "analyze: internal error (row missing in ancestor)"; return ERR_PATTERN; }
          S.tpos.push_back((int32_t)q);
        }
        S.relptr.push_back((int64_t)S.tpos.size());
        int64_t a1 = a;
        while (a1 < r && S.snode_of[R[a1]] == P) {
          S.opair[S.obase[J] + a1] = (int32_t)pid;
          S.ocbase[S.obase[J] + a1] = S.loff[P] + (int64_t(R[a1]) - S.sptr[P]) * mP;
          ++a1;
        }
        a = a1;
      }
    }
    // ---- map of A's entries into supernodal storage ------------------------
    S.amap.resize(nz);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        int64_t a = S.pinv[rowind[p]], b = S.pinv[j];
        int64_t r = std::max(a, b), c = std::min(a, b);
        int64_t J = S.snode_of[c];
        int64_t f = S.sptr[J], k = S.sptr[J + 1] - f, m = S.rptr[J + 1] - S.rptr[J];
        int64_t pos;
        if (r < f + k) {
          pos = r - f;
        } else {
          const int32_t* R = S.rows.data() + S.rptr[J];
          pos = std::lower_bound(R + k, R + m, (int32_t)r) - R;
        }
        S.amap[p] = S.loff[J] + (c - f) * m + pos;
      }
    // ---- full-symmetric CSR of A (original ordering) ----------------------
    S.a_rp.assign(n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        S.a_rp[rowind[p] + 1]++;
        if (rowind[p] != j) S.a_rp[j + 1]++;
      }
    for (int64_t i = 0; i < n; ++i) S.a_rp[i + 1] += S.a_rp[i];
    S.a_col.resize(S.a_rp[n]);
    S.a_vidx.resize(S.a_rp[n]);
    {
      // row i gets (i, j) for the lower entries of row i (j <= i, from the
      // columns j in increasing order) and then (i, r) for the entries of
      // column i below the diagonal: columns ascend within each row
      std::vector<int64_t> fill(S.a_rp.begin(), S.a_rp.end() - 1);
      for (int64_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
          const int64_t i = rowind[p];
          S.a_col[fill[i]] = (int32_t)j;
          S.a_vidx[fill[i]++] = p;
        }
      for (int64_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j] + 1; p < colptr[j + 1]; ++p) {
          S.a_col[fill[j]] = (int32_t)rowind[p];
          S.a_vidx[fill[j]++] = p;
        }
    }
    // ---- levels --------------------------------------------------------
    S.level.assign(ns, 0);
    for (int64_t J = 0; J < ns; ++J)
      if (S.sparent[J] >= 0) S.level[S.sparent[J]] = std::max(S.level[S.sparent[J]], S.level[J] + 1);
    S.nlevels = 0;
    for (int64_t J = 0; J < ns; ++J) S.nlevels = std::max(S.nlevels, S.level[J] + 1);
    // ---- launch schedule ------------------------------------------------
    std::vector<std::vector<int32_t>> bylev(S.nlevels);
    for (int64_t J = 0; J < ns; ++J) bylev[S.level[J]].push_back((int32_t)J);
    auto K = [&](int64_t J) { return S.sptr[J + 1] - S.sptr[J]; };
    auto M = [&](int64_t J) { return S.rptr[J + 1] - S.rptr[J]; };
    auto npan = [&](int64_t J) { return (K(J) + nb - 1) / nb; };
    auto kpan = [&](int64_t J, int64_t p) { return std::min<int64_t>(nb, K(J) - p * nb); };
    auto open = [&](std::vector<Launch>& plan, int32_t kind, int32_t lev, int32_t pan) {
      Launch L;
      L.kind = kind; L.ntasks = 0; L.off = (int64_t)S.tasks.size(); L.level = lev; L.panel = pan;
      plan.push_back(L);
    };
    // lower-triangle entries (i >= c) of rows [r0, r1) x cols [c0, c1)
    auto lower_count = [](int64_t r0, int64_t r1, int64_t c0, int64_t c1) {
      int64_t s = 0;
      for (int64_t c = c0; c < c1; ++c) s += std::max<int64_t>(0, r1 - std::max(r0, c));
      return s;
    };
    // algorithmic flops and HBM bytes of one task (solves: per right-hand side)
    auto cost = [&](int32_t kind, const Task& t, double& fl, double& by) {
      const int64_t J = t.J, k = K(J), m = M(J);
      switch (kind) {
        case K_SMALL: {
          // factor and solve of all K columns, the inverse block, the update
          // of the r rows below (r (r + 1) / 2 scattered entries)
          const int64_t r = m - k;
          for (int64_t j = 0; j < k; ++j) fl += double(k - j) * double(k - j);
          fl += double(r) * double(k) * double(k) + double(k) * double(k) * double(k) / 3.0;
          fl += 2.0 * double(k) * double(r * (r + 1) / 2);
          by += 16.0 * double(k * m) + 8.0 * double(k * (k + 1) / 2) + 16.0 * double(r * (r + 1) / 2);
          break;
        }
        case K_MEDIUM: {
          // factor of the K columns, the inverse block, the r rows below solved
          const int64_t r = m - k;
          for (int64_t j = 0; j < k; ++j) fl += double(k - j) * double(k - j);
          fl += double(r) * double(k) * double(k) + double(k) * double(k) * double(k) / 3.0;
          by += 16.0 * double(k * m) + 8.0 * double(k * (k + 1) / 2);
          break;
        }
        case K_FACTOR:
        case K_TRSM: {
          const int64_t c0 = int64_t(t.a) * nb, kp = std::min<int64_t>(nb, k - c0);
          const bool diag = kind == K_FACTOR;
          const int64_t rb = t.b, re = std::min<int64_t>(t.b + (diag ? kTrsmRows : kTile), m);
          const int64_t nr = std::max<int64_t>(0, re - rb);
          if (diag) {
            for (int64_t j = 0; j < kp; ++j) fl += double(kp - j) * double(kp - j);
            by += 16.0 * double(kp * (kp + 1) / 2);
            if (t.c == 1) {  // update of the diagonal block by the previous panel
              fl += 2.0 * double(nb) * double(kp * (kp + 1) / 2);
              by += 8.0 * double(nb) * double(kp);
            } else if (t.c >= 3) {
              // the block's rows in panel p-1: (c = 4: panel p-2's update,)
              // the solve with W_{p-1} (read, triangle), the rows written; the
              // diagonal block's update by one or two panels
              const double np = t.c == 4 ? 2.0 : 1.0;
              if (t.c == 4) {
                fl += 2.0 * double(nb) * double(nb) * double(kp);
                by += 16.0 * double(nb) * double(kp);
              }
              fl += double(kp) * double(nb) * double(nb) + np * 2.0 * double(nb) * double(kp * (kp + 1) / 2);
              by += 16.0 * double(nb) * double(kp) + 8.0 * double(nb * (nb + 1) / 2);
            }
          } else {
            by += 8.0 * double(kp * (kp + 1) / 2);
            if (t.c == 1) {  // the previous panel's update of the tile, its rows of both panels read
              const int64_t kq = std::min<int64_t>(nb, k - c0);
              fl += 2.0 * double(nb) * double(nr) * double(kq);
              by += 8.0 * double(nb) * double(nr + kq);
            }
          }
          fl += double(nr) * double(kp) * double(kp);
          by += 16.0 * double(nr * kp);
          break;
        }
        case K_UPD_INT:
        case K_UPD_EXT: {
          const bool range = kind == K_UPD_INT && (t.c & kPanelRange);
          const int64_t kb = kind == K_UPD_INT ? int64_t(range ? (t.c & 0xffff) : t.c) * nb : 0;
          const int64_t kk = kind == K_UPD_INT ? std::min<int64_t>(range ? ((t.c >> 16) & 0xff) * nb : nb, k - kb) : k;
          const int64_t colEnd = kind == K_UPD_INT ? k : m;
          const int64_t r1 = std::min<int64_t>(t.a + kTile, m), c1 = std::min<int64_t>(t.b + kTile, colEnd);
          const int64_t valid = lower_count(t.a, r1, t.b, c1);
          fl += 2.0 * double(kk) * double(valid);
          by += 8.0 * double(kk) * double((r1 - t.a) + (c1 - t.b)) + 16.0 * double(valid);
          break;
        }
        case K_UPD_RLB: {
          const int64_t r0 = t.a & ((1 << 25) - 1), nr = (t.a >> 25) + 1;
          const int64_t c0 = t.b & ((1 << 25) - 1), nc = (t.b >> 25) + 1;
          int64_t valid = 0;
          for (int64_t c = c0; c < c0 + nc; ++c) valid += std::max<int64_t>(0, r0 + nr - std::max(r0, c));
          fl += 2.0 * double(k) * double(valid);
          by += 8.0 * double(k) * double(nr + nc) + 16.0 * double(valid);
          break;
        }
        case K_FWD2: {  // (two-panel tasks; single-panel ones are costed as K_FWD)
            // z_p, the coupling block (kp1 x kp), z_{p+1}; the tile's rows in
            // both panels' columns
            const int64_t kp = std::min<int64_t>(nb, k - int64_t(t.a) * nb);
            const int64_t c1 = int64_t(t.a) * nb + kp, kp1 = std::min<int64_t>(nb, k - c1);
            const int64_t nr = t.b < 0 ? 0 : std::min<int64_t>(t.b + kTile, m) - t.b;
            fl += double(kp) * double(kp) + 2.0 * double(kp1) * double(kp) + double(kp1) * double(kp1) +
                  2.0 * double(nr) * double(kp + kp1);
            by += 8.0 * double(nr) * double(kp + kp1) + 16.0 * double(nr) +
                  ((t.c & 1) ? 8.0 * double(kp * (kp + 1) / 2 + kp1 * (kp1 + 1) / 2 + kp1 * kp) : 0.0);
            break;
          }
        case K_FWD_SMALL:
        case K_BWD_SMALL: {
          const int64_t nr = m - k;
          fl += 2.0 * double(nr) * double(k) + double(k) * double(k);
          by += 8.0 * double(nr) * double(k) + 16.0 * double(nr) + 8.0 * double(k * (k + 1) / 2);
          break;
        }
        case K_FWD:
        case K_BWD: {
          // the rows of L below the panel that the task covers, read once;
          // their entries of y / x; the panel's inverted diagonal block once
          // per panel
          const int64_t kp = std::min<int64_t>(nb, k - int64_t(t.a) * nb);
          int64_t nr = 0;
          bool once = false;
          if (kind == K_FWD || kind == K_FWD2) {
            nr = t.b < 0 ? 0 : std::min<int64_t>(t.b + kTile, m) - t.b;
            once = (t.c & 1) != 0;
          } else {
            nr = t.c < 0 ? m - t.b : (t.c == 0 ? std::min<int64_t>(t.b + kTile, m) - t.b : int64_t(t.c) - 1);
            once = t.c != 0;
          }
          fl += 2.0 * double(nr) * double(kp) + (once ? double(kp) * double(kp) : 0.0);
          by += 8.0 * double(nr) * double(kp) + 16.0 * double(nr) + (once ? 8.0 * double(kp * (kp + 1) / 2) : 0.0);
          break;
        }
        default: break;
      }
    };
    auto close = [&](std::vector<Launch>& plan) {
      Launch& L = plan.back();
      L.ntasks = (int32_t)((int64_t)S.tasks.size() - L.off);
      if (L.ntasks == 0) { plan.pop_back(); return; }
      for (int64_t q = L.off; q < L.off + L.ntasks; ++q) {
        int32_t kind = L.kind;
        if (kind == K_FACTOR_LA)
          kind = q - L.off < L.nfirst ? K_FACTOR : q - L.off < L.nfirst + L.ntrsm ? K_TRSM : K_UPD_INT;
        // a single-panel task of a two-panel forward round does what a K_FWD task does
        if (kind == K_FWD2 && !(S.tasks[q].c & 2)) kind = K_FWD;
        cost(kind, S.tasks[q], L.flops, L.bytes);
      }
    };
    // (SPCHOL_PANEL_ROUNDS=2: the two-launch panel rounds everywhere)
    const char* pr_env = std::getenv("SPCHOL_PANEL_ROUNDS");
    const bool fp_rounds = !(pr_env && std::atoi(pr_env) == 2);
    for (int64_t l = 0; l < S.nlevels; ++l) {
      // supernodes small enough for one wavefront: their whole step in one
      // launch; the panel rounds and tiled updates below take the others
      // then the short one-panel supernodes of at most 32 columns that are
      // not: one wavefront each factors them, their update goes to the
      // external update tiles with the others'
      std::vector<int32_t> lev, upd;
      open(S.factor_plan, K_SMALL, (int32_t)l, -1);
      for (int32_t J : bylev[l]) {
        if (small_supernode(K(J), M(J))) S.tasks.push_back({J, 0, 0, 0});
        else upd.push_back(J);
      }
      close(S.factor_plan);
      // (a launch of its own only when it takes the level's panel rounds
      // away altogether or holds enough tasks to pay for the extra launch)
      int64_t nmed = 0;
      for (int32_t J : upd) nmed += medium_supernode(K(J), M(J), nb);
      const bool med = nmed > 0 && (nmed == (int64_t)upd.size() || nmed >= kMediumMin);
      open(S.factor_plan, K_MEDIUM, (int32_t)l, -1);
      for (int32_t J : upd)
        if (med && medium_supernode(K(J), M(J), nb) && K(J) <= 16) S.tasks.push_back({J, 0, 0, 0});
      S.factor_plan.back().nfirst = (int32_t)((int64_t)S.tasks.size() - S.factor_plan.back().off);
      for (int32_t J : upd) {
        if (med && medium_supernode(K(J), M(J), nb)) {
          if (K(J) > 16) S.tasks.push_back({J, 0, 0, 0});
        } else {
          lev.push_back(J);
        }
      }
      close(S.factor_plan);
      int64_t maxp = 0;
      for (int32_t J : lev) maxp = std::max(maxp, npan(J));
      // internal update tiles of panel p-1 deferred into the launch that
      // factors panel p: the first column tile of the trailing part (which
      // holds panel p) is updated before that launch, the other tiles touch
      // only columns right of panel p and run beside its factorization
      std::vector<Task> deferred;
      // How many rows below the block the diagonal task of round p solves
      // itself: with many tasks in the launch, up to kTrsmRows (parallelism
      // comes from the tasks); with few, none, so that the rows go to the
      // parallel row-tile launch and the diagonal task (the sequential part)
      // stays short -- unless every panel of the launch has at most one tile
      // of rows, when the row-tile launch is skipped altogether.
      std::vector<int64_t> inl_of(maxp + 1, 0);
      for (int64_t p = 0; p < maxp; ++p) {
        int64_t ntask = 0, maxrows = 0;
        for (int32_t J : lev)
          if (npan(J) > p) {
            ++ntask;
            maxrows = std::max<int64_t>(maxrows, M(J) - (p * nb + kpan(J, p)));
          }
        inl_of[p] = ntask >= kInlineMinTasks ? kTrsmRows : (maxrows <= kTile ? kTile : 0);
      }
      // With 64-column panels and no inline rows in round p + 1, the update
      // of panel p + 1's columns by panel p needs no launch of its own: the
      // diagonal task of round p + 1 applies it to its diagonal block first
      // (task field c = 1), the tiles below run beside it
      auto merged = [&](int64_t p) { return nb == kTile && p + 1 < maxp && inl_of[p + 1] == 0; };
      // One launch per panel round (levels of few wide supernodes, whose
      // diagonal tasks solve no rows inline; 64-column panels): round p holds
      //   the diagonal tasks of panel p, which first solve the rows of their
      //     own block in panel p-1's columns (with panel p-2's update of
      //     them) and apply panels p-2 and p-1 to their diagonal block (task
      //     field c = 3: panel p-1 only, c = 4: both);
      //   the row tiles of panel p-1 below those rows (with panel p-2's
      //     update, c = 1);
      //   panel p-2's update tiles of the column blocks from p on (below the
      //     diagonal block in block p).
      // A round's three sets touch disjoint entries and read only entries
      // the rounds before completed; round maxp holds the last row tiles.
      bool one_launch = fp_rounds && nb == kTile && maxp >= 2;
      // (the deterministic schedule has no window: a block entering it would
      // take several atomic ranges in one launch)
      const int64_t win = S.deterministic ? 0 : kRoundWindow;
      for (int64_t p = 0; p < maxp && one_launch; ++p) one_launch = inl_of[p] != kTrsmRows;
      if (one_launch) {
        for (int64_t p = 0; p <= maxp; ++p) {
          open(S.factor_plan, K_FACTOR_LA, (int32_t)l, (int32_t)p);
          for (int32_t J : lev)
            if (npan(J) > p) S.tasks.push_back({J, (int32_t)p, (int32_t)M(J), p == 0 ? 0 : (p == 1 ? 3 : 4)});
          Launch& LL = S.factor_plan.back();
          LL.nfirst = (int32_t)((int64_t)S.tasks.size() - LL.off);
          if (p >= 1)
            for (int32_t J : lev) {
              if (npan(J) <= p - 1) continue;
              const int64_t s0 = npan(J) > p ? p * nb + kpan(J, p) : (p - 1) * nb + kpan(J, p - 1);
              for (int64_t r0 = s0; r0 < M(J); r0 += kTile)
                S.tasks.push_back({J, (int32_t)(p - 1), (int32_t)r0, p - 1 >= 1 ? 1 : 0});
            }
          LL.ntrsm = (int32_t)((int64_t)S.tasks.size() - LL.off) - LL.nfirst;
          // (with a window of D column blocks: panel p-2 goes to blocks p ..
          // p + D - 1 only; block p + D enters the window and takes panels
          // 0 .. p - 2 at once, in ranges of kRangePanels; blocks past it
          // wait)
          if (p >= 2)
            for (int32_t J : lev) {
              const int64_t cend = win > 0 && npan(J) <= 0xffff ? std::min<int64_t>(npan(J), p + win) : npan(J);
              for (int64_t cb = p; cb < cend; ++cb) {
                const int64_t c0 = cb * nb;
                for (int64_t r0 = cb == p ? c0 + kpan(J, p) : c0; r0 < M(J); r0 += kTile)
                  S.tasks.push_back({J, (int32_t)r0, (int32_t)c0, (int32_t)(p - 2)});
              }
              // (a range's first panel is held in 16 bits: no window past that)
              if (win > 0 && p + win < npan(J) && npan(J) <= 0xffff) {
                const int64_t c0 = (p + win) * nb;
                for (int64_t s0 = 0; s0 <= p - 2; s0 += kRangePanels) {
                  const int64_t ns = std::min<int64_t>(kRangePanels, p - 1 - s0);
                  for (int64_t r0 = c0; r0 < M(J); r0 += kTile)
                    S.tasks.push_back({J, (int32_t)r0, (int32_t)c0, (int32_t)(s0 | (ns << 16) | kPanelRange)});
                }
              }
            }
          close(S.factor_plan);
        }
      }
      for (int64_t p = 0; p < maxp && !one_launch; ++p) {
        const int64_t inl = inl_of[p];
        open(S.factor_plan, K_FACTOR, (int32_t)l, (int32_t)p);
        for (int32_t J : lev) {
          if (npan(J) <= p) continue;
          const int64_t rb = p * nb + kpan(J, p);
          // b: first row the task solves inline (== m: none)
          S.tasks.push_back({J, (int32_t)p, (int32_t)(inl > 0 ? rb : M(J)), (p > 0 && merged(p - 1)) ? 1 : 0});
        }
        S.factor_plan.back().nfirst = (int32_t)((int64_t)S.tasks.size() - S.factor_plan.back().off);
        if (!deferred.empty()) {
          S.factor_plan.back().kind = K_FACTOR_LA;
          S.tasks.insert(S.tasks.end(), deferred.begin(), deferred.end());
          deferred.clear();
        }
        close(S.factor_plan);
        open(S.factor_plan, K_TRSM, (int32_t)l, (int32_t)p);
        for (int32_t J : lev) {
          if (npan(J) <= p) continue;
          for (int64_t r0 = p * nb + kpan(J, p) + inl; r0 < M(J); r0 += kTile)
            S.tasks.push_back({J, (int32_t)p, (int32_t)r0, 0});
        }
        close(S.factor_plan);
        open(S.factor_plan, K_UPD_INT, (int32_t)l, (int32_t)p);
        for (int32_t J : lev) {
          if (npan(J) <= p + 1) continue;
          for (int64_t c0 = (p + 1) * nb; c0 < K(J); c0 += kTile)
            for (int64_t r0 = c0; r0 < M(J); r0 += kTile) {
              const Task t{J, (int32_t)r0, (int32_t)c0, (int32_t)p};
              if (c0 != (p + 1) * nb) deferred.push_back(t);
              else if (!merged(p)) S.tasks.push_back(t);
              else if (r0 != c0) deferred.push_back(t);  // (r0 == c0: done by the diagonal task)
            }
        }
        close(S.factor_plan);
      }
      if (!deferred.empty()) {  // (cannot happen: the last panels defer nothing)
        open(S.factor_plan, K_UPD_INT, (int32_t)l, (int32_t)maxp);
        S.tasks.insert(S.tasks.end(), deferred.begin(), deferred.end());
        deferred.clear();
        close(S.factor_plan);
      }
      // external update tiles: those with a target column in the next
      // level run now; the others ("far": every target two or more levels
      // up) go to a second launch marked `side`, which the runtime runs on a
      // second stream beside the next level's panel chain (a chain alone
      // leaves most of the GPU idle) and joins before the level after
      std::vector<Task> far;
      const int32_t ext_kind = S.update_method == 1 ? K_UPD_RLB : K_UPD_EXT;
      open(S.factor_plan, ext_kind, (int32_t)l, -1);
      for (int32_t J : upd) {
        const int32_t* R = S.rows.data() + S.rptr[J];
        if (S.update_method == 1) {
          // RLB (Sec. II-B): J's rows below its columns in blocks of
          // consecutive indices inside one supernode; for every block B (the
          // target columns, in supernode P) and every block B' at or below
          // it, the product L_B'J L_BJ^T goes straight into P's storage at
          // the rows of B' (consecutive there too) and the columns of B:
          // one relative index (the position of B''s first row in P) per
          // block.  Tiles of at most 64 x 64 inside each block pair.
          std::vector<int64_t> bs;  // block starts (local rows), then M(J)
          for (int64_t a = K(J); a < M(J); ++a)
            if (a == K(J) || R[a] != R[a - 1] + 1 || S.snode_of[R[a]] != S.snode_of[R[a - 1]]) bs.push_back(a);
          bs.push_back(M(J));
          S.rlb_blocks += (int64_t)bs.size() - 1;
          for (size_t bi = 0; bi + 1 < bs.size(); ++bi) {
            const int64_t cb = bs[bi], ce = bs[bi + 1];
            const int64_t P = S.snode_of[R[cb]];
            const bool isfar = l + 2 < S.nlevels && !S.deterministic && S.level[P] > l + 1;
            const int32_t* PR = S.rows.data() + S.rptr[P];
            const int64_t mP = S.rptr[P + 1] - S.rptr[P];
            for (size_t bj = bi; bj + 1 < bs.size(); ++bj) {
              const int64_t rb = bs[bj], re = bs[bj + 1];
              const int64_t pos_rb = std::lower_bound(PR, PR + mP, R[rb]) - PR;
              for (int64_t c0 = cb; c0 < ce; c0 += kTile)
                for (int64_t r0 = (bj == bi ? c0 : rb); r0 < re; r0 += kTile) {
                  const int64_t nr = std::min<int64_t>(kTile, re - r0), nc = std::min<int64_t>(kTile, ce - c0);
                  const Task t{J, (int32_t)(r0 | ((nr - 1) << 25)), (int32_t)(c0 | ((nc - 1) << 25)),
                               (int32_t)(pos_rb + (r0 - rb))};
                  if (isfar) far.push_back(t);
                  else S.tasks.push_back(t);
                }
            }
          }
          continue;
        }
        for (int64_t c0 = K(J); c0 < M(J); c0 += kTile) {
          bool isfar = l + 2 < S.nlevels && !S.deterministic;
          for (int64_t c = c0; c < std::min<int64_t>(c0 + kTile, M(J)) && isfar; ++c)
            isfar = S.level[S.snode_of[R[c]]] > l + 1;
          for (int64_t r0 = c0; r0 < M(J); r0 += kTile) {
            const Task t{J, (int32_t)r0, (int32_t)c0, -1};
            if (isfar) far.push_back(t);
            else S.tasks.push_back(t);
          }
        }
      }
      close(S.factor_plan);
      open(S.factor_plan, ext_kind, (int32_t)l, -1);
      S.factor_plan.back().side = 1;
      S.tasks.insert(S.tasks.end(), far.begin(), far.end());
      close(S.factor_plan);
    }
    // forward solve: leaves to root, panels ascending, one launch per round
    // of two panels: a supernode with panels p and p + 1 gets two-panel
    // tasks (c bit 1: z_p, the coupling block's update of panel p + 1's
    // right-hand side, z_{p+1}, then a 64-row tile below panel p + 1 with
    // both), one whose last panel is p single-panel tasks; one task per
    // 64-row tile (c bit 0 on the first, which also stores the solution);
    // no rows below: one task with b = -1
    // Small one-panel supernodes of a level that holds many of them get a
    // launch of their own (one wavefront each) in both solves; `rest` is the
    // level without them.
    std::vector<std::vector<int32_t>> rest(S.nlevels), smalls(S.nlevels);
    for (int64_t l = 0; l < S.nlevels; ++l) {
      for (int32_t J : bylev[l])
        (small_solve_supernode(K(J), M(J), nb) ? smalls[l] : rest[l]).push_back(J);
      if ((int64_t)smalls[l].size() < kSmallSolveMin) {
        rest[l] = bylev[l];
        smalls[l].clear();
      }
    }
    // (the supernodes with at most 64 rows below first: nfirst of them)
    auto small_launch = [&](std::vector<Launch>& plan, int32_t kind, int64_t l) {
      if (smalls[l].empty()) return;
      open(plan, kind, (int32_t)l, 0);
      for (int32_t J : smalls[l])
        if (M(J) - K(J) <= kTile) S.tasks.push_back({J, 0, (int32_t)K(J), 1});
      plan.back().nfirst = (int32_t)((int64_t)S.tasks.size() - plan.back().off);
      for (int32_t J : smalls[l])
        if (M(J) - K(J) > kTile) S.tasks.push_back({J, 0, (int32_t)K(J), 1});
      close(plan);
    };
    for (int64_t l = 0; l < S.nlevels; ++l) {
      small_launch(S.fwd_plan, K_FWD_SMALL, l);
      int64_t maxp = 0;
      for (int32_t J : rest[l]) maxp = std::max(maxp, npan(J));
      for (int64_t p = 0; p < maxp; p += 2) {
        bool two = false;
        for (int32_t J : rest[l]) two = two || npan(J) > p + 1;
        open(S.fwd_plan, two ? K_FWD2 : K_FWD, (int32_t)l, (int32_t)p);
        for (int32_t J : rest[l]) {
          if (npan(J) <= p) continue;
          const bool dbl = npan(J) > p + 1;
          const int64_t below = dbl ? (p + 1) * nb + kpan(J, p + 1) : p * nb + kpan(J, p);
          const int32_t f = dbl ? 2 : 0;
          if (below >= M(J)) S.tasks.push_back({J, (int32_t)p, -1, f | 1});
          for (int64_t r0 = below; r0 < M(J); r0 += kTile)
            S.tasks.push_back({J, (int32_t)p, (int32_t)r0, f | (r0 == below ? 1 : 0)});
        }
        close(S.fwd_plan);
      }
    }
    // backward solve: root to leaves, panels descending, one launch per
    // round.  A panel with at most kBwdRows rows below is done by one task
    // (c = -1: gather, then the inverted diagonal block).  A taller one is
    // split with a one-panel lookahead: its far rows (past the next panel,
    // whose solution is final one round earlier) are added into an
    // accumulator by 64-row tiles (c = 0) in the launch of the round before,
    // and its finishing task (c = 1 + n) gathers the n rows of the next
    // panel, subtracts the accumulator and applies the inverse.  The far
    // tiles of a level's first round run in a launch of their own.
    for (int64_t l = S.nlevels - 1; l >= 0; --l) {
      small_launch(S.bwd_plan, K_BWD_SMALL, l);
      int64_t maxp = 0;
      for (int32_t J : rest[l]) maxp = std::max(maxp, npan(J));
      auto below = [&](int32_t J, int64_t p) { return p * nb + kpan(J, p); };
      // (deterministic: never split, the accumulator would take several adds per entry)
      auto split = [&](int32_t J, int64_t p) {
        return !S.deterministic && p >= 0 && p < npan(J) && M(J) - below(J, p) > kBwdRows;
      };
      auto near = [&](int32_t J, int64_t p) { return p + 1 < npan(J) ? kpan(J, p + 1) : int64_t(0); };
      auto far_tiles = [&](int32_t J, int64_t p) {
        for (int64_t r0 = below(J, p) + near(J, p); r0 < M(J); r0 += kTile)
          S.tasks.push_back({J, (int32_t)p, (int32_t)r0, 0});
      };
      bool pro = false;
      for (int32_t J : rest[l]) pro = pro || split(J, maxp - 1);
      if (pro) {
        open(S.bwd_plan, K_BWD, (int32_t)l, (int32_t)maxp);
        for (int32_t J : rest[l])
          if (split(J, maxp - 1)) far_tiles(J, maxp - 1);
        close(S.bwd_plan);
      }
      for (int64_t p = maxp - 1; p >= 0; --p) {
        open(S.bwd_plan, K_BWD, (int32_t)l, (int32_t)p);
        for (int32_t J : rest[l]) {
          if (npan(J) <= p) continue;
          if (split(J, p)) S.tasks.push_back({J, (int32_t)p, (int32_t)below(J, p), (int32_t)(1 + near(J, p))});
          else S.tasks.push_back({J, (int32_t)p, (int32_t)below(J, p), -1});
        }
        for (int32_t J : rest[l])
          if (split(J, p - 1)) far_tiles(J, p - 1);
        close(S.bwd_plan);
      }
    }
    // selected inversion (reverse mode): root to leaves, last panel first;
    // the panels of one round get slots 0.. (inverse, T) and Y blocks
    for (int64_t l = S.nlevels - 1; l >= 0; --l) {
      int64_t maxp = 0;
      for (int32_t J : bylev[l]) maxp = std::max(maxp, npan(J));
      for (int64_t p = maxp - 1; p >= 0; --p) {
        std::vector<int32_t> js;
        for (int32_t J : bylev[l])
          if (npan(J) > p) js.push_back(J);
        const int64_t base = (int64_t)S.si_yoff.size();
        int64_t yo = 0;
        for (int32_t J : js) {
          S.si_yoff.push_back(yo);
          yo += (M(J) - (p * nb + kpan(J, p))) * kMaxPanel;
        }
        S.si_max_slots = std::max<int64_t>(S.si_max_slots, (int64_t)js.size());
        S.si_max_y = std::max(S.si_max_y, yo);
        // (the inverted diagonal blocks come from the factorization)
        const int32_t kinds[3] = {K_SI_Y, K_SI_ZB, K_SI_ZD};
        for (int32_t kind : kinds) {
          open(S.si_plan, kind, (int32_t)l, (int32_t)p);
          S.si_plan.back().slot_base = base;
          // Y: the segment length of the round.  A task's time grows with its
          // segment (a chain of gathers of Z), so a round of few tasks gets
          // shorter segments, as long as all its tasks still fit the GPU at
          // once; a large round keeps long ones (fewer atomic partial sums)
          int64_t seg = kSiSeg;
          if (kind == K_SI_Y) {
            auto ntasks = [&](int64_t sl) {
              int64_t c = 0;
              for (int32_t J : js) {
                const int64_t r = M(J) - (p * nb + kpan(J, p));
                c += ((r + kTile - 1) / kTile) * ((r + sl - 1) / sl);
              }
              return c;
            };
            while (seg > kTile && ntasks(seg / 2) <= kSiTasksMax) seg /= 2;
            S.si_plan.back().seg = (int32_t)seg;
          }
          for (size_t s = 0; s < js.size(); ++s) {
            const int32_t J = js[s];
            const int64_t rb = p * nb + kpan(J, p);
            if (kind == K_SI_Y) {
              // split K: segments of `seg` rows of B per task (a = panel |
              // segment << 16), summed into the Y blocks (zero on entry:
              // their readers leave them cleared)
              for (int64_t a0 = rb; a0 < M(J); a0 += kTile)
                for (int64_t sg = 0; rb + sg * seg < M(J); ++sg)
                  S.tasks.push_back({J, (int32_t)(p | (sg << 16)), (int32_t)a0, (int32_t)s});
            } else if (kind == K_SI_ZB) {
              for (int64_t a0 = rb; a0 < M(J); a0 += kTile)
                S.tasks.push_back({J, (int32_t)p, (int32_t)a0, (int32_t)s});
            } else {
              S.tasks.push_back({J, (int32_t)p, 0, (int32_t)s});
            }
          }
          Launch& Lb = S.si_plan.back();
          Lb.ntasks = (int32_t)((int64_t)S.tasks.size() - Lb.off);
          if (Lb.ntasks == 0) S.si_plan.pop_back();
        }
      }
    }
    // deterministic schedule: every launch whose tasks add into shared
    // entries (fp64 atomics) is split into launches whose adds hit disjoint
    // entries, run in a fixed order.  Two supernodes of a level add into a
    // common entry (external update, forward solve) exactly when their
    // off-diagonal row lists meet (a common row r gives the common diagonal
    // target (r, r)), so the supernodes of each level are coloured greedily,
    // smallest free colour first, and a launch is split by colour; the
    // selected inversion's Y segments and the T sums of its Z tiles are
    // split by segment and by tile.
    if (S.deterministic) {
      std::vector<int32_t> color(ns, 0);
      {
        std::vector<std::vector<int32_t>> used(n);  // colours holding row r, this level
        std::vector<char> taken;
        for (int64_t l = 0; l < S.nlevels; ++l) {
          for (int32_t J : bylev[l]) {
            const int32_t* R = S.rows.data() + S.rptr[J];
            taken.assign(taken.size(), 0);
            for (int64_t i = K(J); i < M(J); ++i)
              for (int32_t c : used[R[i]]) {
                if ((size_t)c >= taken.size()) taken.resize(c + 1, 0);
                taken[c] = 1;
              }
            int32_t c = 0;
            while ((size_t)c < taken.size() && taken[c]) ++c;
            color[J] = c;
            for (int64_t i = K(J); i < M(J); ++i) used[R[i]].push_back(c);
          }
          for (int32_t J : bylev[l]) {
            const int32_t* R = S.rows.data() + S.rptr[J];
            for (int64_t i = K(J); i < M(J); ++i) used[R[i]].clear();
          }
        }
      }
      auto split_plan = [&](std::vector<Launch>& plan) {
        std::vector<Launch> out;
        for (const Launch& L : plan) {
          int32_t kind = L.kind;
          auto key = [&](const Task& t) -> int64_t {
            if (kind == K_SI_Y) return t.a >> 16;
            if (kind == K_SI_ZB) return t.b;
            return color[t.J];
          };
          const bool adds = kind == K_SMALL || kind == K_UPD_EXT || kind == K_UPD_RLB || kind == K_FWD ||
                            kind == K_FWD2 || kind == K_FWD_SMALL || kind == K_SI_Y || kind == K_SI_ZB;
          if (!adds) { out.push_back(L); continue; }
          Task* t0 = S.tasks.data() + L.off;
          // (small forward solves: within a colour, the supernodes with at
          // most 64 rows below first, nfirst of them per part)
          const bool rows_first = kind == K_FWD_SMALL;
          auto tall = [&](const Task& t) { return rows_first && M(t.J) - K(t.J) > kTile; };
          std::stable_sort(t0, t0 + L.ntasks, [&](const Task& a, const Task& b) {
            return key(a) != key(b) ? key(a) < key(b) : (!tall(a) && tall(b));
          });
          int64_t parts = 0;
          for (int64_t q = 0; q < L.ntasks;) {
            int64_t e = q + 1;
            while (e < L.ntasks && key(t0[e]) == key(t0[q])) ++e;
            Launch P = L;
            P.off = L.off + q;
            P.ntasks = (int32_t)(e - q);
            if (rows_first) {
              P.nfirst = 0;
              for (int64_t u = q; u < e; ++u) P.nfirst += !tall(t0[u]);
            }
            P.flops = P.bytes = 0;
            for (int64_t u = P.off; u < P.off + P.ntasks; ++u) {
              int32_t kd = kind;
              if (kd == K_FWD2 && !(S.tasks[u].c & 2)) kd = K_FWD;
              cost(kd, S.tasks[u], P.flops, P.bytes);
            }
            out.push_back(P);
            ++parts;
            q = e;
          }
          S.max_colors = std::max(S.max_colors, parts);
        }
        plan.swap(out);
      };
      split_plan(S.factor_plan);
      split_plan(S.fwd_plan);
      split_plan(S.si_plan);
    }
    // row and column of each stored entry (original ordering)
    S.e_row.resize(nz);
    S.e_col.resize(nz);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        S.e_row[p] = (int32_t)rowind[p];
        S.e_col[p] = (int32_t)j;
      }
    if (S.tasks.size() >= (size_t(1) << 31)) { err = "analyze: schedule too large"; return ERR_OOM; }
    return 0;
  } catch (const std::bad_alloc&) {
    err = "analyze: out of host memory";
    return ERR_OOM;
  }
}

}  // namespace spchol
