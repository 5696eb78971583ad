// Nested-dissection ordering of a general sparse symmetric pattern: a
// multilevel graph bisection of this library's own, standing in for the
// METIS nested dissection the paper orders its matrices with (Sec. IV-A).
//
//   order(V):  |V| <= leaf: minimum-degree elimination of the subgraph;
//              else split V = A u B u S with no edge between A and B,
//              order(A), order(B), then S (eliminated last).
//   split:     coarsen by heavy-edge matching (vertex and edge weights
//              summed) down to ~400 vertices; bisect the coarsest graph by
//              greedy graph growing from 32 seeds (the cut with the
//              smallest weight within the balance limit); project back
//              level by level, each time improving the cut by
//              Fiduccia-Mattheyses passes (single-vertex moves by gain,
//              best prefix kept, balance kept); the vertex separator is a
//              minimum vertex cover of the bipartite graph of cut edges
//              (Konig: maximum matching by augmenting paths, then the
//              alternating-reachability cover), improved by
//              Fiduccia-Mattheyses moves of separator vertices.
// Parts of more than 20000 vertices keep the smallest separator of three
// independent bisections.  Vertices with equal closed neighbourhoods (the unknowns of one node of a
// system) are first compressed into one weighted vertex.
// Deterministic for a given seed (a splitmix64 stream drives every random
// choice).
#include <algorithm>
#include <climits>
#include <cstdint>
#include <numeric>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "order.hpp"

namespace spchol {

namespace {

struct Rng {
  uint64_t s;
  uint64_t next() {  // splitmix64
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  int64_t below(int64_t n) { return n > 0 ? (int64_t)(next() % (uint64_t)n) : 0; }
};

struct Graph {
  int64_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  std::vector<int64_t> ew;  // edge weights (parallel to adj)
  std::vector<int64_t> vw;  // vertex weights
  int64_t total_vw() const { return std::accumulate(vw.begin(), vw.end(), int64_t(0)); }
};

// Heavy-edge matching: visit vertices in random order, match each unmatched
// vertex with its unmatched neighbour of largest edge weight.  Returns the
// coarse graph and the map fine -> coarse.
Graph coarsen(const Graph& g, Rng& rng, std::vector<int32_t>& cmap) {
  const int64_t n = g.n;
  std::vector<int32_t> order(n), match(n, -1);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t i = n - 1; i > 0; --i) std::swap(order[i], order[rng.below(i + 1)]);
  for (int32_t v : order) {
    if (match[v] >= 0) continue;
    int32_t best = -1;
    int64_t bw = -1;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
      const int32_t u = g.adj[p];
      if (match[u] < 0 && u != v && g.ew[p] > bw) { bw = g.ew[p]; best = u; }
    }
    if (best >= 0) { match[v] = best; match[best] = v; }
    else match[v] = v;
  }
  cmap.assign(n, -1);
  int32_t nc = 0;
  for (int32_t v : order)
    if (cmap[v] < 0) { cmap[v] = nc; cmap[match[v]] = nc; ++nc; }
  Graph c;
  c.n = nc;
  c.vw.assign(nc, 0);
  for (int64_t v = 0; v < n; ++v) c.vw[cmap[v]] += g.vw[v];
  // coarse adjacency: merge the neighbour lists of each matched pair
  std::vector<std::vector<int32_t>> members(nc);
  for (int64_t v = 0; v < n; ++v) members[cmap[v]].push_back((int32_t)v);
  std::vector<int64_t> slot(nc, -1);
  c.xadj.assign(nc + 1, 0);
  for (int32_t cv = 0; cv < nc; ++cv) {
    const int64_t start = (int64_t)c.adj.size();
    for (int32_t v : members[cv])
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
        const int32_t cu = cmap[g.adj[p]];
        if (cu == cv) continue;
        if (slot[cu] >= start) c.ew[slot[cu]] += g.ew[p];
        else { slot[cu] = (int64_t)c.adj.size(); c.adj.push_back(cu); c.ew.push_back(g.ew[p]); }
      }
    c.xadj[cv + 1] = (int64_t)c.adj.size();
  }
  return c;
}

int64_t cut_weight(const Graph& g, const std::vector<char>& side) {
  int64_t w = 0;
  for (int64_t v = 0; v < g.n; ++v)
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
      if (side[v] != side[g.adj[p]]) w += g.ew[p];
  return w / 2;
}

// Greedy graph growing: grow side 1 from `seed` by largest gain (edge weight
// into the grown set minus weight out of it) until it holds half the weight.
std::vector<char> grow(const Graph& g, int32_t seed) {
  const int64_t half = g.total_vw() / 2;
  std::vector<char> side(g.n, 0);
  std::vector<int64_t> gain(g.n, 0);
  std::vector<char> inq(g.n, 0);
  using E = std::pair<int64_t, int32_t>;
  std::priority_queue<E> pq;
  int64_t w = 0;
  auto add = [&](int32_t v) {
    side[v] = 1;
    w += g.vw[v];
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
      const int32_t u = g.adj[p];
      if (side[u]) continue;
      gain[u] += 2 * g.ew[p];
      pq.push({gain[u], u});
      inq[u] = 1;
    }
  };
  for (int64_t v = 0; v < g.n; ++v) {
    int64_t d = 0;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) d += g.ew[p];
    gain[v] = -d;
  }
  add(seed);
  while (w < half) {
    int32_t v = -1;
    while (!pq.empty()) {
      E e = pq.top();
      pq.pop();
      if (!side[e.second] && e.first == gain[e.second]) { v = e.second; break; }
    }
    if (v < 0) {  // disconnected: continue from any vertex outside
      for (int64_t u = 0; u < g.n && v < 0; ++u)
        if (!side[u]) v = (int32_t)u;
      if (v < 0) break;
    }
    add(v);
  }
  return side;
}

// Fiduccia-Mattheyses passes: repeatedly move the boundary vertex of best
// gain to the other side (each vertex once per pass), keep the best prefix
// of moves whose parts stay within the balance limit.
void refine(const Graph& g, std::vector<char>& side, int64_t maxw) {
  const int64_t n = g.n;
  std::vector<int64_t> ext(n), intw(n);
  for (int pass = 0; pass < 8; ++pass) {
    int64_t w1 = 0, total = g.total_vw();
    for (int64_t v = 0; v < n; ++v) w1 += side[v] ? g.vw[v] : 0;
    for (int64_t v = 0; v < n; ++v) {
      ext[v] = intw[v] = 0;
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
        (side[g.adj[p]] != side[v] ? ext[v] : intw[v]) += g.ew[p];
    }
    using E = std::pair<int64_t, int32_t>;
    std::priority_queue<E> pq;
    for (int64_t v = 0; v < n; ++v)
      if (ext[v] > 0) pq.push({ext[v] - intw[v], (int32_t)v});
    std::vector<char> moved(n, 0);
    std::vector<int32_t> seq;
    int64_t cur = 0, best = 0;
    size_t bestlen = 0;
    int fruitless = 0;
    while (!pq.empty() && fruitless < std::max<int64_t>(64, n / 50)) {
      E e = pq.top();
      pq.pop();
      const int32_t v = e.second;
      if (moved[v] || e.first != ext[v] - intw[v]) continue;
      const int64_t nw1 = w1 + (side[v] ? -g.vw[v] : g.vw[v]);
      if (nw1 > maxw || total - nw1 > maxw) continue;
      moved[v] = 1;
      cur += ext[v] - intw[v];
      side[v] ^= 1;
      w1 = nw1;
      seq.push_back(v);
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
        const int32_t u = g.adj[p];
        if (side[u] == side[v]) { intw[u] += g.ew[p]; ext[u] -= g.ew[p]; }
        else { intw[u] -= g.ew[p]; ext[u] += g.ew[p]; }
        if (!moved[u]) pq.push({ext[u] - intw[u], u});
      }
      std::swap(ext[v], intw[v]);
      if (cur > best) { best = cur; bestlen = seq.size(); fruitless = 0; }
      else ++fruitless;
    }
    for (size_t i = seq.size(); i > bestlen; --i) side[seq[i - 1]] ^= 1;  // undo past the best prefix
    if (best <= 0) break;
  }
}

// Bisection of g: multilevel, sides 0 / 1 of roughly equal vertex weight.
std::vector<char> bisect(const Graph& g, Rng& rng) {
  const int64_t total = g.total_vw();
  if (g.n <= 400) {
    std::vector<char> best;
    int64_t bc = -1;
    const int tries = (int)std::min<int64_t>(g.n, 32);
    for (int t = 0; t < tries; ++t) {
      std::vector<char> s = grow(g, (int32_t)rng.below(g.n));
      refine(g, s, total / 2 + std::max<int64_t>(total / 10, 1));
      const int64_t c = cut_weight(g, s);
      if (bc < 0 || c < bc) { bc = c; best = s; }
    }
    return best;
  }
  std::vector<int32_t> cmap;
  Graph c = coarsen(g, rng, cmap);
  std::vector<char> cs;
  if (c.n >= g.n * 19 / 20) {  // matching stalled: bisect this level directly
    std::vector<char> best;
    int64_t bc = -1;
    for (int t = 0; t < 4; ++t) {
      std::vector<char> s = grow(g, (int32_t)rng.below(g.n));
      refine(g, s, total / 2 + std::max<int64_t>(total / 20, 1));
      const int64_t cw = cut_weight(g, s);
      if (bc < 0 || cw < bc) { bc = cw; best = s; }
    }
    return best;
  }
  cs = bisect(c, rng);
  std::vector<char> side(g.n);
  for (int64_t v = 0; v < g.n; ++v) side[v] = cs[cmap[v]];
  refine(g, side, total / 2 + std::max<int64_t>(total / 20, 1));
  return side;
}

// Minimum vertex cover of the bipartite graph of cut edges (Konig).
std::vector<char> separator(const Graph& g, const std::vector<char>& side) {
  const int64_t n = g.n;
  std::vector<int32_t> left;  // boundary vertices of side 0
  std::vector<int32_t> mate(n, -1);
  for (int64_t v = 0; v < n; ++v)
    if (side[v] == 0)
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
        if (side[g.adj[p]] == 1) { left.push_back((int32_t)v); break; }
  // maximum matching by augmenting paths (Kuhn, each search a BFS over
  // alternating paths; par[u] = the left vertex a right vertex was reached from)
  std::vector<int64_t> seen(n, -1);
  std::vector<int32_t> par(n, -1), queue;
  int64_t stamp = 0;
  for (int32_t root : left) {
    if (mate[root] >= 0) continue;
    ++stamp;
    queue.assign(1, root);
    seen[root] = stamp;
    int32_t freeu = -1;
    for (size_t h = 0; h < queue.size() && freeu < 0; ++h) {
      const int32_t v = queue[h];
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
        const int32_t u = g.adj[p];
        if (side[u] != 1 || seen[u] == stamp) continue;
        seen[u] = stamp;
        par[u] = v;
        if (mate[u] < 0) { freeu = u; break; }
        const int32_t w = mate[u];
        if (seen[w] != stamp) { seen[w] = stamp; queue.push_back(w); }
      }
    }
    // augment: flip the alternating path ending at the free right vertex
    for (int32_t u = freeu; u >= 0;) {
      const int32_t l = par[u];
      const int32_t next = mate[l];
      mate[u] = l;
      mate[l] = u;
      u = next;
    }
  }
  // Konig: Z = vertices reachable from unmatched left vertices by
  // alternating paths; cover = (left \ Z) u (right n Z)
  std::vector<char> inz(n, 0);
  queue.clear();
  for (int32_t v : left)
    if (mate[v] < 0) { inz[v] = 1; queue.push_back(v); }
  for (size_t h = 0; h < queue.size(); ++h) {
    const int32_t v = queue[h];
    if (side[v] == 0) {
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
        const int32_t u = g.adj[p];
        if (side[u] == 1 && !inz[u] && mate[v] != u) { inz[u] = 1; queue.push_back(u); }
      }
    } else if (mate[v] >= 0 && !inz[mate[v]]) {
      inz[mate[v]] = 1;
      queue.push_back(mate[v]);
    }
  }
  std::vector<char> sep(n, 0);
  for (int32_t v : left)
    if (!inz[v]) sep[v] = 1;
  for (int64_t v = 0; v < n; ++v)
    if (side[v] == 1 && inz[v]) {
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
        if (side[g.adj[p]] == 0) { sep[v] = 1; break; }
    }
  return sep;
}

// Vertex-separator refinement (Fiduccia-Mattheyses on the separator): a
// separator vertex moved into part X pulls its neighbours in the other part
// into the separator; gain = its weight minus theirs.  Moves by best gain
// (stale gains recomputed when popped), each vertex once per pass, parts
// within maxw, the best prefix of a pass kept.  label: 0 / 1 parts, 2 the
// separator.
void refine_separator(const Graph& g, std::vector<char>& label, int64_t maxw) {
  const int64_t n = g.n;
  auto gain = [&](int32_t v, int x) {  // move v (in the separator) into part x
    int64_t pulled = 0;
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
      if (label[g.adj[p]] == 1 - x) pulled += g.vw[g.adj[p]];
    return g.vw[v] - pulled;
  };
  for (int pass = 0; pass < 8; ++pass) {
    int64_t w[3] = {0, 0, 0};
    for (int64_t v = 0; v < n; ++v) w[(int)label[v]] += g.vw[v];
    using E = std::tuple<int64_t, int32_t, int>;
    std::priority_queue<E> pq;
    for (int64_t v = 0; v < n; ++v)
      if (label[v] == 2)
        for (int x = 0; x < 2; ++x) pq.push({gain((int32_t)v, x), (int32_t)v, x});
    std::vector<char> locked(n, 0);
    struct Move { int32_t v; int x; std::vector<int32_t> pulled; };
    std::vector<Move> seq;
    int64_t cur = 0, best = 0;
    size_t bestlen = 0;
    int64_t fruitless = 0;
    const int64_t limit = std::max<int64_t>(64, n / 50);
    while (!pq.empty() && fruitless < limit) {
      auto [gv, v, x] = pq.top();
      pq.pop();
      if (label[v] != 2 || locked[v]) continue;
      const int64_t gnow = gain(v, x);
      if (gnow != gv) { pq.push({gnow, v, x}); continue; }
      int64_t pulled_w = 0;
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p)
        if (label[g.adj[p]] == 1 - x) pulled_w += g.vw[g.adj[p]];
      if (w[x] + g.vw[v] > maxw) continue;
      Move mv{v, x, {}};
      label[v] = (char)x;
      locked[v] = 1;
      w[x] += g.vw[v];
      w[2] -= g.vw[v];
      for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) {
        const int32_t u = g.adj[p];
        if (label[u] == 1 - x) {
          label[u] = 2;
          w[1 - x] -= g.vw[u];
          w[2] += g.vw[u];
          mv.pulled.push_back(u);
          if (!locked[u]) pq.push({gain(u, x), u, x}), pq.push({gain(u, 1 - x), u, 1 - x});
        }
      }
      cur += gnow;
      seq.push_back(std::move(mv));
      if (cur > best) { best = cur; bestlen = seq.size(); fruitless = 0; }
      else ++fruitless;
      (void)pulled_w;
    }
    for (size_t i = seq.size(); i > bestlen; --i) {  // undo past the best prefix
      const Move& mv = seq[i - 1];
      for (int32_t u : mv.pulled) label[u] = (char)(1 - mv.x);
      label[mv.v] = 2;
    }
    if (best <= 0) break;
  }
}

// Induced subgraph of the weighted graph (xadj, adj, ew, vw) on `verts`.
Graph induced(const Graph& w, const std::vector<int32_t>& verts, std::vector<int32_t>& local) {
  Graph g;
  g.n = (int64_t)verts.size();
  for (size_t i = 0; i < verts.size(); ++i) local[verts[i]] = (int32_t)i;
  g.xadj.assign(g.n + 1, 0);
  g.vw.resize(g.n);
  for (size_t i = 0; i < verts.size(); ++i) {
    const int32_t v = verts[i];
    g.vw[i] = w.vw[v];
    for (int64_t p = w.xadj[v]; p < w.xadj[v + 1]; ++p)
      if (local[w.adj[p]] >= 0) { g.adj.push_back(local[w.adj[p]]); g.ew.push_back(w.ew[p]); }
    g.xadj[i + 1] = (int64_t)g.adj.size();
  }
  for (int32_t v : verts) local[v] = -1;
  return g;
}

// Minimum-degree elimination of a small subgraph (explicit elimination graph).
void min_degree(const Graph& g, const std::vector<int32_t>& verts, std::vector<int64_t>& out) {
  const int64_t n = g.n;
  std::vector<std::vector<int32_t>> nb(n);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t p = g.xadj[v]; p < g.xadj[v + 1]; ++p) nb[v].push_back(g.adj[p]);
  std::vector<char> done(n, 0);
  for (int64_t step = 0; step < n; ++step) {
    int64_t best = -1;
    for (int64_t v = 0; v < n; ++v)
      if (!done[v] && (best < 0 || nb[v].size() < nb[best].size())) best = v;
    done[best] = 1;
    out.push_back(verts[best]);
    // the neighbours of best become a clique
    std::vector<int32_t> nbrs;
    for (int32_t u : nb[best])
      if (!done[u]) nbrs.push_back(u);
    for (int32_t u : nbrs) {
      std::vector<int32_t> merged;
      for (int32_t w : nb[u])
        if (!done[w]) merged.push_back(w);
      for (int32_t w : nbrs)
        if (w != u) merged.push_back(w);
      std::sort(merged.begin(), merged.end());
      merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
      nb[u].swap(merged);
    }
  }
}

}  // namespace

int order_nd(int64_t n, const int64_t* colptr, const int64_t* rowind, int64_t leaf, uint64_t seed, int64_t* perm,
             std::string& err) {
  try {
    if (n < 0 || !colptr || (n > 0 && (!rowind || !perm))) { err = "order_nd: null pointer or n < 0"; return -1; }
    if (n >= (int64_t(1) << 31) - 1) { err = "order_nd: n too large"; return -1; }
    if (leaf < 1) leaf = 64;
    // symmetric adjacency without the diagonal or duplicates
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t j = 0; j < n; ++j)
      for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
        const int64_t i = rowind[p];
        if (i < 0 || i >= n) { err = "order_nd: row index out of range"; return -2; }
        if (i != j) { deg[i + 1]++; deg[j + 1]++; }
      }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> adj0(deg[n]);
    {
      std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
      for (int64_t j = 0; j < n; ++j)
        for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
          const int64_t i = rowind[p];
          if (i != j) { adj0[fill[i]++] = (int32_t)j; adj0[fill[j]++] = (int32_t)i; }
        }
    }
    std::vector<int64_t> xadj(n + 1, 0);
    std::vector<int32_t> adj;
    adj.reserve(adj0.size());
    for (int64_t v = 0; v < n; ++v) {
      std::sort(adj0.begin() + deg[v], adj0.begin() + deg[v + 1]);
      for (int64_t p = deg[v]; p < deg[v + 1]; ++p)
        if (p == deg[v] || adj0[p] != adj0[p - 1]) adj.push_back(adj0[p]);
      xadj[v + 1] = (int64_t)adj.size();
    }
    std::vector<int32_t>().swap(adj0);
    // Compression: vertices with the same closed neighbourhood (the dofs of
    // one node of a system, say) are indistinguishable to every separator
    // and elimination order; they become one vertex of that weight and are
    // eliminated together, in increasing original index.
    std::vector<int32_t> grp(n, -1);
    std::vector<std::vector<int32_t>> members;
    {
      std::vector<uint64_t> h(n);
      for (int64_t v = 0; v < n; ++v) {  // a sum over the closed neighbourhood, and the degree
        uint64_t sum = (uint64_t)v * 0xD6E8FEB86659FD93ULL;
        for (int64_t p = xadj[v]; p < xadj[v + 1]; ++p) sum += (uint64_t)adj[p] * 0xD6E8FEB86659FD93ULL;
        h[v] = sum ^ ((uint64_t)(xadj[v + 1] - xadj[v]) << 48);
      }
      std::vector<int32_t> idx(n);
      std::iota(idx.begin(), idx.end(), 0);
      std::sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return h[a] != h[b] ? h[a] < h[b] : a < b; });
      auto same = [&](int32_t a, int32_t b) {  // closed neighbourhoods equal
        if (xadj[a + 1] - xadj[a] != xadj[b + 1] - xadj[b]) return false;
        // adj(a) u {a} == adj(b) u {b}: b in adj(a), and the rest agree
        int64_t pa = xadj[a], pb = xadj[b];
        const int64_t ea = xadj[a + 1], eb = xadj[b + 1];
        bool ba = false, ab = false;
        while (pa < ea || pb < eb) {
          int32_t va = pa < ea ? adj[pa] : INT32_MAX, vb = pb < eb ? adj[pb] : INT32_MAX;
          if (va == b) { ba = true; ++pa; continue; }
          if (vb == a) { ab = true; ++pb; continue; }
          if (va != vb) return false;
          ++pa;
          ++pb;
        }
        return ba && ab;
      };
      for (int64_t s0 = 0; s0 < n;) {
        int64_t e0 = s0 + 1;
        while (e0 < n && h[idx[e0]] == h[idx[s0]]) ++e0;
        for (int64_t a = s0; a < e0; ++a) {
          const int32_t va = idx[a];
          if (grp[va] >= 0) continue;
          grp[va] = (int32_t)members.size();
          members.push_back({va});
          for (int64_t b = a + 1; b < e0; ++b) {
            const int32_t vb = idx[b];
            if (grp[vb] < 0 && same(va, vb)) { grp[vb] = grp[va]; members.back().push_back(vb); }
          }
        }
        s0 = e0;
      }
    }
    const int64_t nc = (int64_t)members.size();
    Graph cg;  // compressed graph
    cg.n = nc;
    cg.vw.resize(nc);
    cg.xadj.assign(nc + 1, 0);
    {
      std::vector<int64_t> seen(nc, -1);
      for (int64_t c = 0; c < nc; ++c) {
        std::sort(members[c].begin(), members[c].end());
        cg.vw[c] = (int64_t)members[c].size();
        const int32_t v = members[c][0];
        for (int64_t p = xadj[v]; p < xadj[v + 1]; ++p) {
          const int32_t d = grp[adj[p]];
          if (d == c || seen[d] == c) continue;
          seen[d] = c;
          cg.adj.push_back(d);
          cg.ew.push_back((int64_t)members[c].size());  // times |d|, set below
        }
        cg.xadj[c + 1] = (int64_t)cg.adj.size();
      }
      for (int64_t c = 0; c < nc; ++c)
        for (int64_t p = cg.xadj[c]; p < cg.xadj[c + 1]; ++p) cg.ew[p] *= (int64_t)members[cg.adj[p]].size();
    }
    std::vector<int32_t>().swap(adj);
    Rng rng{seed ? seed : 0x5EEDULL};
    std::vector<int32_t> local(nc, -1);
    std::vector<int64_t> out;  // compressed vertices in elimination order
    out.reserve(nc);
    // explicit stack of (vertex set, separator to append after it)
    struct Item {
      std::vector<int32_t> verts;
      bool emit;  // true: append verts as they are (a separator)
    };
    std::vector<Item> stack;
    std::vector<int32_t> all(nc);
    std::iota(all.begin(), all.end(), 0);
    stack.push_back({std::move(all), false});
    while (!stack.empty()) {
      Item it = std::move(stack.back());
      stack.pop_back();
      if (it.emit) {
        out.insert(out.end(), it.verts.begin(), it.verts.end());
        continue;
      }
      if (it.verts.empty()) continue;
      Graph g = induced(cg, it.verts, local);
      if ((int64_t)it.verts.size() <= leaf) {
        min_degree(g, it.verts, out);
        continue;
      }
      // large parts: the smallest separator of a few independent
      // multilevel bisections (the top separators decide most of the fill)
      const int tries = g.n > 20000 ? 3 : 1;
      std::vector<char> label;
      int64_t best_w = -1;
      for (int t = 0; t < tries; ++t) {
        std::vector<char> side = bisect(g, rng);
        std::vector<char> sep = separator(g, side);
        std::vector<char> lab(g.n);
        for (int64_t v = 0; v < g.n; ++v) lab[v] = sep[v] ? 2 : side[v];
        refine_separator(g, lab, g.total_vw() / 2 + std::max<int64_t>(g.total_vw() / 20, 1));
        int64_t sw = 0;
        for (int64_t v = 0; v < g.n; ++v) sw += lab[v] == 2 ? g.vw[v] : 0;
        if (best_w < 0 || sw < best_w) { best_w = sw; label.swap(lab); }
      }
      std::vector<int32_t> A, B, Sv;
      for (int64_t v = 0; v < g.n; ++v) {
        if (label[v] == 2) Sv.push_back(it.verts[v]);
        else (label[v] ? B : A).push_back(it.verts[v]);
      }
      if (A.empty() || B.empty()) {  // no useful split (a clique-like piece)
        min_degree(g, it.verts, out);
        continue;
      }
      // order A, then B, then the separator: push in reverse
      stack.push_back({std::move(Sv), true});
      stack.push_back({std::move(B), false});
      stack.push_back({std::move(A), false});
    }
    if ((int64_t)out.size() != nc) { err = "order_nd: internal error (ordering incomplete)"; return -2; }
    int64_t k = 0;
    for (int64_t c : out)
      for (int32_t v : members[c]) perm[k++] = v;
    if (k != n) { err = "order_nd: internal error (expansion incomplete)"; return -2; }
    return 0;
  } catch (const std::bad_alloc&) {
    err = "order_nd: out of host memory";
    return -4;
  }
}

}  // namespace spchol
