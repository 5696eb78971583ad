/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for supernodal
 * sparse Cholesky.  TEST INFRASTRUCTURE ONLY: the GPU library never links,
 * includes or calls anything in this directory, and this file includes
 * nothing from the library.
 *
 * What it computes (all in fp64, single thread, no BLAS):
 *
 *   structure  Column structures of L for C = P A P^T by set unions
 *              (Sec. II: the structure of column j minus j is contained in
 *              the structure of its parent, and the parent is the smallest
 *              off-diagonal row of column j):
 *                struct(L_j) = {j} u {i > j : C_ij != 0}
 *                              u  U_{c : parent(c) = j} struct(L_c) \ {c}.
 *              Supernodes (Sec. I, Sec. II-A): runs of consecutive columns
 *              with equal structure below the diagonal ("maximal"), and in
 *              the "fundamental" mode additionally each column is the only
 *              etree child of the next.  Relaxed amalgamation (Sec. IV-A
 *              merges a supernode with its parent; the acceptance rule here
 *              is the "<= z explicit zeros per column" rule of the 3D
 *              workloads), or the greedy rule of Sec. IV-A: repeatedly the
 *              merge adding the least new storage, up to a cap on the
 *              cumulative increase).  Supernodal etree (Fig. 1).  Relative indices
 *              relind(J, P) (Sec. II-A, the distance of a row from the
 *              bottom of P's row list; the positional reading of the
 *              worked example of Fig. 1).
 *   numeric    The unique lower-triangular L with positive diagonal and
 *              C = L L^T (Sec. II), by a plain left-looking column
 *              algorithm with a dense accumulator, and (cross-check) by an
 *              up-looking row algorithm.
 *   solve      y = L^{-1} P b, z = L^{-T} y, x = P^T z.
 *   logdet     2 * sum_j log L_jj with pairwise summation.
 *
 * Conventions: 0-based indices; input A is the lower triangle incl. the
 * diagonal in CSC, rows strictly increasing within a column; perm[k] is the
 * original index eliminated k-th (NULL = identity).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n;
  int64_t nnzA;
  int64_t *pinv;           /* pinv[original] = permuted index */
  int64_t *cptr, *crow;    /* C = P A P^T, lower, by column, rows sorted */
  int64_t *cmap;           /* cmap[p] = position in crow of A's entry p */
  int64_t *parent;         /* column etree */
  int64_t *count;          /* c_j = |struct(L_j)| incl. diagonal */
  int64_t *lptr, *lrow;    /* struct(L) by column, diagonal first */
  int64_t nsuper;
  int64_t *sptr;           /* nsuper+1: first column of each supernode */
  int64_t *sparent;        /* supernodal etree parent, -1 for roots */
  int64_t *srptr, *srow;   /* row list of each supernode, sorted */
  int64_t npairs;          /* (J, P) pairs: J updates ancestor P */
  int64_t *pJ, *pP, *pa0;  /* pa0 = index into J's off-diagonal rows */
  int64_t *relptr;
  int32_t *rel;
} osym;

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

void oracle_free(osym *s) {
  if (!s) return;
  free(s->pinv); free(s->cptr); free(s->crow); free(s->cmap);
  free(s->parent); free(s->count); free(s->lptr); free(s->lrow);
  free(s->sptr); free(s->sparent); free(s->srptr); free(s->srow);
  free(s->pJ); free(s->pP); free(s->pa0); free(s->relptr); free(s->rel);
  free(s);
}

/* Growable int64 array. */
typedef struct { int64_t *a; int64_t n, cap; } vec;
static int vpush(vec *v, int64_t x) {
  if (v->n == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 1024;
    int64_t *na = (int64_t *)realloc(v->a, (size_t)nc * sizeof(int64_t));
    if (!na) return -1;
    v->a = na; v->cap = nc;
  }
  v->a[v->n++] = x;
  return 0;
}

/* Permute the lower pattern: entry (i, j) of A goes to
 * (max(pinv i, pinv j), min(...)) of C. */
static int build_C(osym *s, const int64_t *colptr, const int64_t *rowind) {
  int64_t n = s->n, nz = colptr[n];
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t *er = (int64_t *)malloc((size_t)(nz ? nz : 1) * sizeof(int64_t));
  int64_t *ec = (int64_t *)malloc((size_t)(nz ? nz : 1) * sizeof(int64_t));
  if (!cnt || !er || !ec) { free(cnt); free(er); free(ec); return -4; }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p) {
      int64_t i = rowind[p];
      int64_t a = s->pinv[i], b = s->pinv[j];
      er[p] = a > b ? a : b;
      ec[p] = a > b ? b : a;
      cnt[ec[p] + 1]++;
    }
  s->cptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  s->crow = (int64_t *)malloc((size_t)(nz ? nz : 1) * sizeof(int64_t));
  s->cmap = (int64_t *)malloc((size_t)(nz ? nz : 1) * sizeof(int64_t));
  if (!s->cptr || !s->crow || !s->cmap) { free(cnt); free(er); free(ec); return -4; }
  s->cptr[0] = 0;
  for (int64_t j = 0; j < n; ++j) s->cptr[j + 1] = s->cptr[j] + cnt[j + 1];
  int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  memcpy(fill, s->cptr, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t p = 0; p < nz; ++p) {
    int64_t q = fill[ec[p]]++;
    s->crow[q] = er[p];
    s->cmap[p] = q;
  }
  /* sort rows inside each column, carrying the map (insertion sort on
   * (row, source) pairs: columns are short) */
  int64_t *src = (int64_t *)malloc((size_t)(nz ? nz : 1) * sizeof(int64_t));
  for (int64_t p = 0; p < nz; ++p) src[s->cmap[p]] = p;
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t a = s->cptr[j] + 1; a < s->cptr[j + 1]; ++a) {
      int64_t r = s->crow[a], sr = src[a], b = a - 1;
      while (b >= s->cptr[j] && s->crow[b] > r) {
        s->crow[b + 1] = s->crow[b]; src[b + 1] = src[b]; --b;
      }
      s->crow[b + 1] = r; src[b + 1] = sr;
    }
    for (int64_t a = s->cptr[j] + 1; a < s->cptr[j + 1]; ++a)
      if (s->crow[a] == s->crow[a - 1]) { free(cnt); free(er); free(ec); free(fill); free(src); return -2; }
    if (s->cptr[j] == s->cptr[j + 1] || s->crow[s->cptr[j]] != j) {
      /* missing diagonal */
      free(cnt); free(er); free(ec); free(fill); free(src); return -2;
    }
  }
  for (int64_t a = 0; a < nz; ++a) s->cmap[src[a]] = a;
  free(src); free(cnt); free(er); free(ec); free(fill);
  return 0;
}

/* Column structures by set unions, in column order. */
static int build_L(osym *s) {
  int64_t n = s->n;
  s->parent = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  s->count = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  s->lptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t *mark = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *chead = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *cnext = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *tmp = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  if (!s->parent || !s->count || !s->lptr || !mark || !chead || !cnext || !tmp) return -4;
  for (int64_t j = 0; j < n; ++j) { mark[j] = -1; chead[j] = -1; }
  vec L = {0, 0, 0};
  s->lptr[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    int64_t t = 0;
    mark[j] = j; tmp[t++] = j;
    for (int64_t p = s->cptr[j]; p < s->cptr[j + 1]; ++p) {
      int64_t i = s->crow[p];
      if (mark[i] != j) { mark[i] = j; tmp[t++] = i; }
    }
    for (int64_t c = chead[j]; c != -1; c = cnext[c]) {
      for (int64_t p = s->lptr[c]; p < s->lptr[c + 1]; ++p) {
        int64_t i = L.a[p];
        if (i == c) continue;
        if (mark[i] != j) { mark[i] = j; tmp[t++] = i; }
      }
    }
    qsort(tmp, (size_t)t, sizeof(int64_t), cmp_i64);
    for (int64_t a = 0; a < t; ++a) if (vpush(&L, tmp[a])) return -4;
    s->lptr[j + 1] = L.n;
    s->count[j] = t;
    s->parent[j] = t > 1 ? tmp[1] : -1;
    if (t > 1) { int64_t pj = tmp[1]; cnext[j] = chead[pj]; chead[pj] = j; }
  }
  s->lrow = L.a ? L.a : (int64_t *)malloc(sizeof(int64_t));
  free(mark); free(chead); free(cnext); free(tmp);
  return 0;
}

/* Does struct(L_j) \ {j} equal struct(L_{j+1})? */
static int same_below(const osym *s, int64_t j) {
  int64_t a0 = s->lptr[j] + 1, a1 = s->lptr[j + 1];
  int64_t b0 = s->lptr[j + 1], b1 = s->lptr[j + 2];
  if (a1 - a0 != b1 - b0) return 0;
  for (int64_t t = 0; t < a1 - a0; ++t)
    if (s->lrow[a0 + t] != s->lrow[b0 + t]) return 0;
  return 1;
}

/* sorted union of two sorted lists into out (returns length) */
static int64_t merge_union(const int64_t *a, int64_t na, const int64_t *b, int64_t nb, int64_t *out) {
  int64_t i = 0, j = 0, k = 0;
  while (i < na || j < nb) {
    if (j >= nb || (i < na && a[i] < b[j])) out[k++] = a[i++];
    else if (i >= na || b[j] < a[i]) out[k++] = b[j++];
    else { out[k++] = a[i++]; ++j; }
  }
  return k;
}

/* storage of a dense lower trapezoid of k columns and m rows */
static int64_t trapezoid(int64_t k, int64_t m) {
  int64_t t = 0;
  for (int64_t c = 0; c < k; ++c) t += m - c;
  return t;
}

/* A binary min-heap of merge candidates (cost, first column, group end,
 * stamp), ordered by cost, then first column. */
typedef struct { int64_t cost, first, end, stamp; } cand;
typedef struct { cand *a; int64_t n, cap; } cheap;

static int cand_less(const cand *x, const cand *y) {
  return x->cost < y->cost || (x->cost == y->cost && x->first < y->first);
}

static void heap_push(cheap *h, cand c) {
  if (h->n == h->cap) {
    h->cap = h->cap ? 2 * h->cap : 64;
    h->a = (cand *)realloc(h->a, (size_t)h->cap * sizeof(cand));
  }
  int64_t i = h->n++;
  h->a[i] = c;
  while (i > 0 && cand_less(&h->a[i], &h->a[(i - 1) / 2])) {
    cand t = h->a[i]; h->a[i] = h->a[(i - 1) / 2]; h->a[(i - 1) / 2] = t;
    i = (i - 1) / 2;
  }
}

static cand heap_pop(cheap *h) {
  cand top = h->a[0];
  h->a[0] = h->a[--h->n];
  for (int64_t i = 0;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && cand_less(&h->a[l], &h->a[m])) m = l;
    if (r < h->n && cand_less(&h->a[r], &h->a[m])) m = r;
    if (m == i) break;
    cand t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
    i = m;
  }
  return top;
}

/* The group holding base supernode b: groups are runs of base supernodes
 * ending at their one alive member, so it is the first alive base from b
 * on (nxt links dead bases forward). */
static int64_t group_of(int64_t *nxt, int64_t b) {
  int64_t r = b;
  while (nxt[r] != r) r = nxt[r];
  while (nxt[b] != r && b != r) { int64_t t = nxt[b]; nxt[b] = r; b = t; }
  return r;
}

/* Push the candidate of group e -- its merge into the group holding its
 * parent column -- if that group starts right after it. */
static void push_candidate(cheap *h, const osym *s, int64_t e, int64_t *nxt, const int64_t *bptr,
                           const int64_t *bsn, int64_t **brows, const int64_t *bm, const int64_t *gfirst,
                           const int64_t *stamp, int64_t *u) {
  const int64_t pc = s->parent[bptr[e + 1] - 1];
  if (pc < 0) return;
  const int64_t q = group_of(nxt, bsn[pc]);
  if (gfirst[q] != bptr[e + 1]) return;
  const int64_t m = merge_union(brows[e], bm[e], brows[q], bm[q], u);
  const int64_t ke = bptr[e + 1] - gfirst[e], kq = bptr[q + 1] - gfirst[q];
  cand c = {trapezoid(ke + kq, m) - trapezoid(ke, bm[e]) - trapezoid(kq, bm[q]), gfirst[e], e, stamp[e]};
  heap_push(h, c);
}

/* The greedy rule (Sec. IV-A): repeatedly merge the pair (group, group
 * holding its parent column) whose merge adds the least new storage
 * (explicit zeros of the merged trapezoid), if the parent group starts
 * right after it; ties go to the group with the smaller first column; stop
 * before the cumulative increase would pass cap_percent of nnz(L).  The
 * cost of a candidate is counted from the explicit union of both row
 * lists.  A merge changes two candidates: the merged group's own and that
 * of the group ending right before it; they are pushed again with a new
 * stamp, older entries are skipped. */
static void greedy_merge(osym *s, int64_t nb, const int64_t *bptr, const int64_t *bsn, int64_t **brows,
                         int64_t *bm, int64_t *gfirst, int64_t *alive, int64_t cap_percent) {
  const int64_t n = s->n;
  int64_t nnzl = 0;
  for (int64_t j = 0; j < n; ++j) nnzl += s->count[j];
  const int64_t cap = nnzl * cap_percent / 100;
  int64_t added = 0;
  int64_t *u = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *nxt = (int64_t *)malloc(((size_t)nb + 1) * sizeof(int64_t));
  int64_t *stamp = (int64_t *)calloc((size_t)(nb ? nb : 1), sizeof(int64_t));
  for (int64_t b = 0; b <= nb; ++b) nxt[b] = b;
  cheap h = {NULL, 0, 0};
  for (int64_t e = 0; e < nb; ++e) push_candidate(&h, s, e, nxt, bptr, bsn, brows, bm, gfirst, stamp, u);
  while (h.n > 0) {
    cand c = heap_pop(&h);
    const int64_t e = c.end;
    if (!alive[e] || c.stamp != stamp[e]) continue;  /* stale */
    if (added + c.cost > cap) break;
    const int64_t q = group_of(nxt, bsn[s->parent[bptr[e + 1] - 1]]);
    int64_t *w = (int64_t *)malloc((size_t)(bm[e] + bm[q]) * sizeof(int64_t));
    int64_t m = merge_union(brows[e], bm[e], brows[q], bm[q], w);
    free(brows[q]);
    brows[q] = w; bm[q] = m; gfirst[q] = gfirst[e];
    alive[e] = 0;
    nxt[e] = e + 1;
    added += c.cost;
    ++stamp[q];
    push_candidate(&h, s, q, nxt, bptr, bsn, brows, bm, gfirst, stamp, u);
    if (gfirst[q] > 0) {
      const int64_t pe = group_of(nxt, bsn[gfirst[q] - 1]);
      ++stamp[pe];
      push_candidate(&h, s, pe, nxt, bptr, bsn, brows, bm, gfirst, stamp, u);
    }
  }
  free(h.a); free(stamp); free(nxt); free(u);
}

static int build_supernodes(osym *s, int mode, int64_t z, int rule, int64_t cap_percent) {
  int64_t n = s->n;
  /* base partition */
  int64_t *nchild = (int64_t *)calloc((size_t)(n ? n : 1), sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j) if (s->parent[j] >= 0) nchild[s->parent[j]]++;
  int64_t *bptr = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t nb = 0;
  for (int64_t j = 0; j < n; ++j) {
    int join = 0;
    if (j > 0 && s->parent[j - 1] == j && same_below(s, j - 1)) {
      join = (mode == 1) ? 1 : (nchild[j] == 1);
    }
    if (!join) bptr[nb++] = j;
  }
  bptr[nb] = n;
  free(nchild);
  /* rows of a column range = union of its columns' structures */
  int64_t *mark = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *tmp = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) mark[i] = -1;
  /* per base supernode: row list */
  int64_t **brows = (int64_t **)calloc((size_t)(nb ? nb : 1), sizeof(int64_t *));
  int64_t *bm = (int64_t *)calloc((size_t)(nb ? nb : 1), sizeof(int64_t));
  int64_t *bsn = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  for (int64_t b = 0; b < nb; ++b) {
    int64_t t = 0;
    for (int64_t j = bptr[b]; j < bptr[b + 1]; ++j) {
      bsn[j] = b;
      for (int64_t p = s->lptr[j]; p < s->lptr[j + 1]; ++p) {
        int64_t i = s->lrow[p];
        if (mark[i] != b) { mark[i] = b; tmp[t++] = i; }
      }
    }
    qsort(tmp, (size_t)t, sizeof(int64_t), cmp_i64);
    brows[b] = (int64_t *)malloc((size_t)(t ? t : 1) * sizeof(int64_t));
    memcpy(brows[b], tmp, (size_t)t * sizeof(int64_t));
    bm[b] = t;
  }
  /* relaxed amalgamation: visit base supernodes in increasing order; try to
   * merge the group ending at s into its parent p when p starts right after
   * s ends.  Merged rows = union of both row lists; accept when the merged
   * storage has at most z explicit zeros per column. */
  int64_t *gfirst = (int64_t *)malloc((size_t)(nb ? nb : 1) * sizeof(int64_t));
  int64_t *alive = (int64_t *)malloc((size_t)(nb ? nb : 1) * sizeof(int64_t));
  for (int64_t b = 0; b < nb; ++b) { gfirst[b] = bptr[b]; alive[b] = 1; }
  if (rule == 1) {
    greedy_merge(s, nb, bptr, bsn, brows, bm, gfirst, alive, cap_percent);
  } else if (z > 0) {
    for (int64_t b = 0; b < nb; ++b) {
      int64_t last = bptr[b + 1] - 1;
      int64_t pc = s->parent[last];
      if (pc < 0) continue;
      int64_t p = bsn[pc];
      if (bptr[p] != last + 1) continue;
      int64_t *u = (int64_t *)malloc((size_t)(bm[b] + bm[p]) * sizeof(int64_t));
      int64_t m = merge_union(brows[b], bm[b], brows[p], bm[p], u);
      int64_t k = bptr[p + 1] - gfirst[b];
      int64_t storage = 0, truenz = 0;
      for (int64_t t = 0; t < k; ++t) storage += m - t;
      for (int64_t j = gfirst[b]; j < bptr[p + 1]; ++j) truenz += s->count[j];
      if (storage - truenz <= z * k) {
        free(brows[p]);
        brows[p] = u; bm[p] = m; gfirst[p] = gfirst[b];
        alive[b] = 0;
      } else {
        free(u);
      }
    }
  }
  /* final supernodes */
  int64_t ns = 0;
  for (int64_t b = 0; b < nb; ++b) ns += alive[b];
  s->nsuper = ns;
  s->sptr = (int64_t *)malloc(((size_t)ns + 1) * sizeof(int64_t));
  s->srptr = (int64_t *)malloc(((size_t)ns + 1) * sizeof(int64_t));
  int64_t tot = 0, q = 0;
  for (int64_t b = 0; b < nb; ++b) if (alive[b]) { s->sptr[q++] = gfirst[b]; tot += bm[b]; }
  s->sptr[ns] = n;
  s->srow = (int64_t *)malloc((size_t)(tot ? tot : 1) * sizeof(int64_t));
  s->srptr[0] = 0; q = 0;
  for (int64_t b = 0; b < nb; ++b) if (alive[b]) {
    memcpy(s->srow + s->srptr[q], brows[b], (size_t)bm[b] * sizeof(int64_t));
    s->srptr[q + 1] = s->srptr[q] + bm[b];
    ++q;
  }
  /* supernode of each column, supernodal parent */
  int64_t *sn = bsn; /* reuse */
  for (int64_t J = 0; J < ns; ++J)
    for (int64_t j = s->sptr[J]; j < s->sptr[J + 1]; ++j) sn[j] = J;
  s->sparent = (int64_t *)malloc((size_t)(ns ? ns : 1) * sizeof(int64_t));
  for (int64_t J = 0; J < ns; ++J) {
    int64_t pc = s->parent[s->sptr[J + 1] - 1];
    s->sparent[J] = pc < 0 ? -1 : sn[pc];
  }
  /* relative indices: for J and each distinct supernode P holding one of J's
   * off-diagonal rows, from the first such row onwards:
   * rel = m_P - 1 - position of the row in P's row list */
  vec vJ = {0, 0, 0}, vP = {0, 0, 0}, va0 = {0, 0, 0}, vptr = {0, 0, 0}, vrel = {0, 0, 0};
  vpush(&vptr, 0);
  for (int64_t J = 0; J < ns; ++J) {
    int64_t m = s->srptr[J + 1] - s->srptr[J];
    int64_t k = s->sptr[J + 1] - s->sptr[J];
    const int64_t *R = s->srow + s->srptr[J] + k;
    int64_t r = m - k;
    int64_t prevP = -1;
    for (int64_t a = 0; a < r; ++a) {
      int64_t P = sn[R[a]];
      if (P == prevP) continue;
      prevP = P;
      const int64_t *PR = s->srow + s->srptr[P];
      int64_t mP = s->srptr[P + 1] - s->srptr[P];
      vpush(&vJ, J); vpush(&vP, P); vpush(&va0, a);
      for (int64_t c = a; c < r; ++c) {
        /* binary search R[c] in P's rows */
        int64_t lo = 0, hi = mP;
        while (lo < hi) { int64_t mid = (lo + hi) / 2; if (PR[mid] < R[c]) lo = mid + 1; else hi = mid; }
        if (lo >= mP || PR[lo] != R[c]) { return -2; }
        vpush(&vrel, mP - 1 - lo);
      }
      vpush(&vptr, vrel.n);
    }
  }
  s->npairs = vJ.n;
  s->pJ = vJ.a; s->pP = vP.a; s->pa0 = va0.a; s->relptr = vptr.a;
  s->rel = (int32_t *)malloc((size_t)(vrel.n ? vrel.n : 1) * sizeof(int32_t));
  for (int64_t t = 0; t < vrel.n; ++t) s->rel[t] = (int32_t)vrel.a[t];
  free(vrel.a);
  for (int64_t b = 0; b < nb; ++b) free(brows[b]);
  free(brows); free(bm); free(bsn); free(bptr); free(gfirst); free(alive); free(mark); free(tmp);
  return 0;
}

/* status: 0 ok, -1 bad argument, -2 bad pattern, -4 out of memory */
osym *oracle_symbolic(int64_t n, const int64_t *colptr, const int64_t *rowind,
                      const int64_t *perm, int32_t snode_mode, int64_t amalg_z,
                      int32_t amalg_rule, int64_t amalg_cap_percent, int64_t *status) {
  *status = 0;
  if (n < 0 || !colptr || (n > 0 && !rowind)) { *status = -1; return NULL; }
  osym *s = (osym *)calloc(1, sizeof(osym));
  s->n = n;
  s->nnzA = colptr[n];
  s->pinv = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) s->pinv[i] = -1;
  for (int64_t k = 0; k < n; ++k) {
    int64_t o = perm ? perm[k] : k;
    if (o < 0 || o >= n || s->pinv[o] != -1) { *status = -1; oracle_free(s); return NULL; }
    s->pinv[o] = k;
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = colptr[j]; p < colptr[j + 1]; ++p)
      if (rowind[p] < j || rowind[p] >= n || (p > colptr[j] && rowind[p] <= rowind[p - 1])) {
        *status = -2; oracle_free(s); return NULL;
      }
  int rc = build_C(s, colptr, rowind);
  if (!rc) rc = build_L(s);
  if (!rc) rc = build_supernodes(s, snode_mode, amalg_z, amalg_rule, amalg_cap_percent);
  if (rc) { *status = rc; oracle_free(s); return NULL; }
  return s;
}

/* sizes: n, nnz(L), nsuper, total supernode rows, npairs, total relind */
void oracle_sym_sizes(const osym *s, int64_t *out) {
  out[0] = s->n;
  out[1] = s->lptr[s->n];
  out[2] = s->nsuper;
  out[3] = s->srptr[s->nsuper];
  out[4] = s->npairs;
  out[5] = s->relptr[s->npairs];
}

#define CP(dst, src, cnt, T) do { if (dst) memcpy(dst, src, (size_t)(cnt) * sizeof(T)); } while (0)
void oracle_sym_get(const osym *s, int64_t *pinv, int64_t *parent, int64_t *count, int64_t *lptr,
                    int64_t *lrow, int64_t *sptr, int64_t *sparent, int64_t *srptr, int64_t *srow,
                    int64_t *pJ, int64_t *pP, int64_t *pa0, int64_t *relptr, int32_t *rel) {
  int64_t n = s->n, ns = s->nsuper, np = s->npairs;
  CP(pinv, s->pinv, n, int64_t);
  CP(parent, s->parent, n, int64_t);
  CP(count, s->count, n, int64_t);
  CP(lptr, s->lptr, n + 1, int64_t);
  CP(lrow, s->lrow, s->lptr[n], int64_t);
  CP(sptr, s->sptr, ns + 1, int64_t);
  CP(sparent, s->sparent, ns, int64_t);
  CP(srptr, s->srptr, ns + 1, int64_t);
  CP(srow, s->srow, s->srptr[ns], int64_t);
  CP(pJ, s->pJ, np, int64_t);
  CP(pP, s->pP, np, int64_t);
  CP(pa0, s->pa0, np, int64_t);
  CP(relptr, s->relptr, np + 1, int64_t);
  CP(rel, s->rel, s->relptr[np], int32_t);
}

/* Permuted lower values of C, in the order of (cptr, crow). */
static double *permuted_values(const osym *s, const double *vals) {
  double *cv = (double *)malloc((size_t)(s->nnzA ? s->nnzA : 1) * sizeof(double));
  if (!cv) return NULL;
  for (int64_t p = 0; p < s->nnzA; ++p) cv[s->cmap[p]] = vals[p];
  return cv;
}

/* Left-looking column Cholesky.  Column j: accumulate x = C_{j:n,j} minus
 * L_{j:n,k} L_jk for every earlier column k with L_jk != 0, then
 * L_jj = sqrt(x_j) and L_ij = x_i / L_jj.  The columns k with L_jk != 0 are
 * found with per-row linked lists of "next row to be touched" pointers.
 * Returns 0, or 1 + the first column whose pivot is not positive. */
static int64_t factor_left(const osym *s, const double *cv, double *lv, int64_t ncols) {
  int64_t n = s->n;
  double *x = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  int64_t *head = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *link = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *nextp = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j) head[j] = -1;
  int64_t info = 0;
  for (int64_t j = 0; j < ncols && !info; ++j) {
    for (int64_t p = s->cptr[j]; p < s->cptr[j + 1]; ++p) x[s->crow[p]] += cv[p];
    int64_t k = head[j];
    while (k != -1) {
      int64_t knext = link[k];
      int64_t p = nextp[k];
      double ljk = lv[p];
      for (int64_t q = p; q < s->lptr[k + 1]; ++q) x[s->lrow[q]] -= lv[q] * ljk;
      nextp[k] = p + 1;
      if (p + 1 < s->lptr[k + 1]) {
        int64_t r = s->lrow[p + 1];
        link[k] = head[r]; head[r] = k;
      }
      k = knext;
    }
    double d = x[j];
    if (!(d > 0.0)) { info = j + 1; break; }
    double ljj = sqrt(d);
    lv[s->lptr[j]] = ljj;
    x[j] = 0.0;
    for (int64_t p = s->lptr[j] + 1; p < s->lptr[j + 1]; ++p) {
      int64_t i = s->lrow[p];
      lv[p] = x[i] / ljj;
      x[i] = 0.0;
    }
    if (s->lptr[j] + 1 < s->lptr[j + 1]) {
      nextp[j] = s->lptr[j] + 1;
      int64_t r = s->lrow[s->lptr[j] + 1];
      link[j] = head[r]; head[r] = j;
    }
  }
  free(x); free(head); free(link); free(nextp);
  return info;
}

/* Up-looking row Cholesky (cross-check): row i solves
 * L_{0:i,0:i} l = C_{i,0:i}^T by forward substitution over the row's
 * structure, then L_ii = sqrt(C_ii - l.l). */
static int64_t factor_up(const osym *s, const double *cv, double *lv) {
  int64_t n = s->n, nz = s->lptr[n];
  /* row structure of L (strictly lower), rows ascending, by transposition */
  int64_t *rptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = s->lptr[j] + 1; p < s->lptr[j + 1]; ++p) rptr[s->lrow[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
  int64_t *rcol = (int64_t *)malloc((size_t)((nz - n) > 0 ? (nz - n) : 1) * sizeof(int64_t));
  int64_t *f = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  memcpy(f, rptr, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = s->lptr[j] + 1; p < s->lptr[j + 1]; ++p) rcol[f[s->lrow[p]]++] = j;
  /* transposed C (row access): C row i = entries (i, j) j <= i */
  int64_t nzc = s->cptr[n];
  int64_t *tptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t p = 0; p < nzc; ++p) tptr[s->crow[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  int64_t *tcol = (int64_t *)malloc((size_t)(nzc ? nzc : 1) * sizeof(int64_t));
  double *tval = (double *)malloc((size_t)(nzc ? nzc : 1) * sizeof(double));
  memcpy(f, tptr, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = s->cptr[j]; p < s->cptr[j + 1]; ++p) {
      int64_t q = f[s->crow[p]]++;
      tcol[q] = j; tval[q] = cv[p];
    }
  int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  for (int64_t j = 0; j < n; ++j) fill[j] = s->lptr[j] + 1;
  double *x = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  int64_t info = 0;
  for (int64_t i = 0; i < n && !info; ++i) {
    double cii = 0.0;
    for (int64_t p = tptr[i]; p < tptr[i + 1]; ++p) {
      if (tcol[p] == i) cii = tval[p]; else x[tcol[p]] = tval[p];
    }
    double d = cii;
    for (int64_t t = rptr[i]; t < rptr[i + 1]; ++t) {
      int64_t j = rcol[t];
      double y = x[j] / lv[s->lptr[j]];
      x[j] = 0.0;
      for (int64_t p = s->lptr[j] + 1; p < fill[j]; ++p) x[s->lrow[p]] -= lv[p] * y;
      lv[fill[j]++] = y;
      d -= y * y;
    }
    if (!(d > 0.0)) { info = i + 1; break; }
    lv[s->lptr[i]] = sqrt(d);
  }
  free(rptr); free(rcol); free(f); free(tptr); free(tcol); free(tval); free(fill); free(x);
  return info;
}

/* variant 0: left-looking, 1: up-looking.  lv has nnz(L) entries in the
 * order of (lptr, lrow).  Returns 0 or 1-based failing (permuted) column;
 * -1 on allocation failure.  ncols >= 0 (left-looking only) stops after the
 * first ncols columns: column j depends only on columns k < j, so those
 * columns are final (the rest of lv stays zero). */
int64_t oracle_factor(const osym *s, const double *vals, int32_t variant, int64_t ncols, double *lv) {
  double *cv = permuted_values(s, vals);
  if (!cv) return -1;
  memset(lv, 0, (size_t)s->lptr[s->n] * sizeof(double));
  if (ncols < 0 || ncols > s->n) ncols = s->n;
  int64_t info = variant == 1 ? factor_up(s, cv, lv) : factor_left(s, cv, lv, ncols);
  free(cv);
  return info;
}

/* In place: B (n x nrhs, column-major, leading dimension ldb, original
 * ordering) <- A^{-1} B. */
void oracle_solve(const osym *s, const double *lv, double *B, int64_t nrhs, int64_t ldb) {
  int64_t n = s->n;
  double *y = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
  for (int64_t c = 0; c < nrhs; ++c) {
    double *b = B + c * ldb;
    for (int64_t i = 0; i < n; ++i) y[s->pinv[i]] = b[i];
    for (int64_t j = 0; j < n; ++j) {
      y[j] /= lv[s->lptr[j]];
      for (int64_t p = s->lptr[j] + 1; p < s->lptr[j + 1]; ++p) y[s->lrow[p]] -= lv[p] * y[j];
    }
    for (int64_t j = n - 1; j >= 0; --j) {
      double t = y[j];
      for (int64_t p = s->lptr[j] + 1; p < s->lptr[j + 1]; ++p) t -= lv[p] * y[s->lrow[p]];
      y[j] = t / lv[s->lptr[j]];
    }
    for (int64_t i = 0; i < n; ++i) b[i] = y[s->pinv[i]];
  }
  free(y);
}

static double pairwise(const double *v, int64_t n) {
  if (n <= 8) { double t = 0.0; for (int64_t i = 0; i < n; ++i) t += v[i]; return t; }
  int64_t h = n / 2;
  return pairwise(v, h) + pairwise(v + h, n - h);
}

double oracle_logdet(const osym *s, const double *lv) {
  int64_t n = s->n;
  double *lg = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
  for (int64_t j = 0; j < n; ++j) lg[j] = log(lv[s->lptr[j]]);
  double r = 2.0 * pairwise(lg, n);
  free(lg);
  return r;
}

/* Algorithmic flops sum_{j < ncols} c_j^2 (column Cholesky with sqrt
 * counted once; ncols < 0 = all columns). */
double oracle_flops(const osym *s, int64_t ncols) {
  double f = 0.0;
  if (ncols < 0 || ncols > s->n) ncols = s->n;
  for (int64_t j = 0; j < ncols; ++j) f += (double)s->count[j] * (double)s->count[j];
  return f;
}
