/*
 * Graphlet counting oracle: plain, slow, single-threaded CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes (the paper's problem definition, Section 2 "Notation and
 * Definitions"): for k = 2, 3, 4, the number of k-node subsets of V whose
 * induced subgraph (Definition "Induced Graphlet") is isomorphic to each
 * graphlet of Table 1: 2 + 4 + 11 = 17 classes, connected and disconnected.
 * Output order: g2_1 g2_2 | g3_1..g3_4 | g4_1..g4_11, as numbered in Table 1.
 * Counts are exact unsigned 128-bit integers.
 *
 * Three routes, none sharing code with the others:
 *
 *   oracle_bruteforce      the definition itself: every 2-, 3- and 4-subset
 *                          is classified by the Table 1 columns (edge count
 *                          from the density rho, max degree Delta, number of
 *                          components |C|).  Feasible for n up to a few
 *                          hundred.
 *
 *   oracle_vertex_bruteforce  the same enumeration, crediting each subset to
 *                          its members: per-vertex counts by definition.
 *
 *   oracle_identity_route  exact at any size, by a route the paper does not
 *                          use: counts of NON-induced copies of each
 *                          connected pattern (paths, stars, triangles,
 *                          cycles, diamonds, tailed triangles, cliques) are
 *                          turned into induced counts by inverting the
 *                          "how many copies of H sit on the vertex set of H'"
 *                          matrix, and the disconnected classes come from
 *                          counting (pattern, extra vertex) pairs.  Pinned
 *                          against oracle_bruteforce on random small graphs.
 *
 *   oracle_edge_local      per edge, the 4-subsets containing it split by
 *                          graphlet and by the edge's place in it (the
 *                          N_{a,b,0/1} terms of Section 4.2), by vertex types;
 *                          oracle_edge_local_brute gets the same vector by
 *                          classifying every subset (Table 1) and reading
 *                          the edge's place from degrees.
 *
 *   oracle_per_edge        the per-edge quantities of the paper written out
 *                          literally for one edge at a time: |Tri_e|
 *                          (Section 3, triangles), the number of 4-cliques
 *                          containing e (Corollary "cliq": pairs of Tri_e
 *                          that are adjacent) and the number of induced
 *                          4-cycles containing e (Corollary "cyc": adjacent
 *                          pairs (w, r) with w in Star_u, r in Star_v).
 *
 * Input contract for every entry point: CSR with n rows, row_ptr[n+1],
 * col[row_ptr[n]], neighbour lists strictly increasing, symmetric, no
 * self-loops (the paper drops loops, weights and direction, Section 5).
 * Functions return 0 on success, a negative value on bad input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

typedef struct {
  uint64_t lo, hi;
} orc_u128;

static void put(orc_u128 *o, u128 v) {
  o->lo = (uint64_t)v;
  o->hi = (uint64_t)(v >> 64);
}

static u128 choose(u128 n, int k) {
  /* C(n, k) for k <= 4, exact: each partial product is divisible as written. */
  if (k == 0) return 1;
  if (n < (u128)k) return 0;
  u128 r = 1;
  for (int i = 0; i < k; i++) r = r * (n - i) / (u128)(i + 1);
  return r;
}

/* Checks the CSR contract; 0 if it holds. */
int oracle_check_csr(int64_t n, const int32_t *rp, const int32_t *col) {
  if (n < 0 || rp[0] != 0) return -1;
  for (int64_t u = 0; u < n; u++) {
    if (rp[u + 1] < rp[u]) return -1;
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
      int64_t v = col[j];
      if (v < 0 || v >= n || v == u) return -2;
      if (j > rp[u] && col[j - 1] >= v) return -3;
    }
  }
  /* symmetry: v in N(u) implies u in N(v) (binary search) */
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) {
      int64_t v = col[j];
      int64_t lo = rp[v], hi = rp[v + 1];
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] < u) lo = mid + 1; else hi = mid;
      }
      if (lo == rp[v + 1] || col[lo] != u) return -4;
    }
  return 0;
}

static int adjacent(const int32_t *rp, const int32_t *col, int64_t a, int64_t b) {
  int64_t lo = rp[a], hi = rp[a + 1];
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (col[mid] < b) lo = mid + 1; else hi = mid;
  }
  return lo < rp[a + 1] && col[lo] == b;
}

/* ------------------------------------------------------------------------ */
/* Route 1: brute force over all subsets (the definition).                   */
/* ------------------------------------------------------------------------ */

/*
 * Table 1, 4-node rows: (edges = rho * 6, Delta, |C|) -> index within k=4.
 *   g4_1  4-clique            rho 1.00 -> 6 edges, Delta 3, |C| 1
 *   g4_2  4-chordalcycle      rho 0.83 -> 5 edges, Delta 3, |C| 1
 *   g4_3  4-tailedtriangle    rho 0.67 -> 4 edges, Delta 3, |C| 1
 *   g4_4  4-cycle             rho 0.67 -> 4 edges, Delta 2, |C| 1
 *   g4_5  3-star              rho 0.50 -> 3 edges, Delta 3, |C| 1
 *   g4_6  4-path              rho 0.50 -> 3 edges, Delta 2, |C| 1
 *   g4_7  4-node-1-triangle   rho 0.50 -> 3 edges, Delta 2, |C| 2
 *   g4_8  4-node-2-star       rho 0.33 -> 2 edges, Delta 2, |C| 2
 *   g4_9  4-node-2-edge       rho 0.33 -> 2 edges, Delta 1, |C| 2
 *   g4_10 4-node-1-edge       rho 0.17 -> 1 edge,  Delta 1, |C| 3
 *   g4_11 4-node-independent  rho 0.00 -> 0 edges, Delta 0, |C| 4
 * Returns 0..10 for g4_1..g4_11, or -1 if no row matches.
 */
int oracle_classify4(int edges, int maxdeg, int comps) {
  static const int rows[11][3] = {{6, 3, 1}, {5, 3, 1}, {4, 3, 1}, {4, 2, 1},
                                  {3, 3, 1}, {3, 2, 1}, {3, 2, 2}, {2, 2, 2},
                                  {2, 1, 2}, {1, 1, 3}, {0, 0, 4}};
  for (int i = 0; i < 11; i++)
    if (rows[i][0] == edges && rows[i][1] == maxdeg && rows[i][2] == comps) return i;
  return -1;
}

/* Table 1, 3-node rows: g3_1 triangle (3 edges), g3_2 2-star (2),
 * g3_3 3-node-1-edge (1), g3_4 3-node-independent (0). */
static int classify3(int edges) { return 3 - edges; }

/* Connected components of the induced subgraph on k <= 4 vertices given as a
 * k x k 0/1 matrix (union-find on at most 4 elements). */
static int components(int k, int a[4][4]) {
  int parent[4];
  for (int i = 0; i < k; i++) parent[i] = i;
  for (int i = 0; i < k; i++)
    for (int j = i + 1; j < k; j++)
      if (a[i][j]) {
        int ri = i, rj = j;
        while (parent[ri] != ri) ri = parent[ri];
        while (parent[rj] != rj) rj = parent[rj];
        if (ri != rj) parent[ri] = rj;
      }
  int c = 0;
  for (int i = 0; i < k; i++)
    if (parent[i] == i) c++;
  return c;
}

int oracle_bruteforce(int64_t n, const int32_t *rp, const int32_t *col, orc_u128 out[17]) {
  if (oracle_check_csr(n, rp, col)) return -1;
  if (n > 2000) return -2; /* the dense matrix below is n^2 bytes */
  unsigned char *A = (unsigned char *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1), 1);
  if (!A) return -3;
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) A[u * n + col[j]] = 1;
  u128 c[17];
  memset(c, 0, sizeof c);
  /* k = 2: g2_1 edge, g2_2 2-node-independent */
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++) c[A[a * n + b] ? 0 : 1]++;
  /* k = 3 */
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++)
      for (int64_t d = b + 1; d < n; d++) {
        int e = A[a * n + b] + A[a * n + d] + A[b * n + d];
        c[2 + classify3(e)]++;
      }
  /* k = 4 */
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++)
      for (int64_t d = b + 1; d < n; d++)
        for (int64_t f = d + 1; f < n; f++) {
          int64_t v[4] = {a, b, d, f};
          int m4[4][4];
          int deg[4] = {0, 0, 0, 0}, edges = 0;
          for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
              m4[i][j] = (i != j) && A[v[i] * n + v[j]];
              deg[i] += m4[i][j];
            }
          for (int i = 0; i < 4; i++) edges += deg[i];
          edges /= 2;
          int mx = 0;
          for (int i = 0; i < 4; i++) mx = deg[i] > mx ? deg[i] : mx;
          int cls = oracle_classify4(edges, mx, components(4, m4));
          if (cls < 0) { free(A); return -4; }
          c[6 + cls]++;
        }
  free(A);
  for (int i = 0; i < 17; i++) put(&out[i], c[i]);
  return 0;
}

/*
 * Per-vertex counts by the definition: out[v * 17 + c] is the number of
 * k-subsets S of V with v in S whose induced subgraph is graphlet c (Table 1
 * classes, output order as above).  Every 2-, 3- and 4-subset is classified
 * once and credited to each of its members, so summed over v the column of a
 * k-node class is k times its global count.  Counts fit int64 for the sizes
 * this enumeration can reach (n <= 2000 here).
 */
int oracle_vertex_bruteforce(int64_t n, const int32_t *rp, const int32_t *col, int64_t *out) {
  if (oracle_check_csr(n, rp, col)) return -1;
  if (n > 2000) return -2;
  unsigned char *A = (unsigned char *)calloc((size_t)(n > 0 ? n : 1) * (size_t)(n > 0 ? n : 1), 1);
  if (!A) return -3;
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++) A[u * n + col[j]] = 1;
  memset(out, 0, sizeof(int64_t) * 17 * (size_t)n);
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++) {
      const int c = A[a * n + b] ? 0 : 1;
      out[a * 17 + c]++;
      out[b * 17 + c]++;
    }
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++)
      for (int64_t d = b + 1; d < n; d++) {
        const int c = 2 + classify3(A[a * n + b] + A[a * n + d] + A[b * n + d]);
        out[a * 17 + c]++;
        out[b * 17 + c]++;
        out[d * 17 + c]++;
      }
  for (int64_t a = 0; a < n; a++)
    for (int64_t b = a + 1; b < n; b++)
      for (int64_t d = b + 1; d < n; d++)
        for (int64_t f = d + 1; f < n; f++) {
          int64_t v[4] = {a, b, d, f};
          int m4[4][4];
          int deg[4] = {0, 0, 0, 0}, edges = 0, mx = 0;
          for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
              m4[i][j] = (i != j) && A[v[i] * n + v[j]];
              deg[i] += m4[i][j];
            }
          for (int i = 0; i < 4; i++) {
            edges += deg[i];
            mx = deg[i] > mx ? deg[i] : mx;
          }
          const int cls = oracle_classify4(edges / 2, mx, components(4, m4));
          if (cls < 0) {
            free(A);
            return -4;
          }
          for (int i = 0; i < 4; i++) out[v[i] * 17 + 6 + cls]++;
        }
  free(A);
  return 0;
}

/*
 * Per-edge brute force for tiny graphs: for each listed edge (u, v), the
 * number of 4-subsets {u, v, w, r} inducing a 4-clique and the number
 * inducing a 4-cycle (chordless, 4 edges, max degree 2).
 */
int oracle_bruteforce_edge4(int64_t n, const int32_t *rp, const int32_t *col, int64_t cnt,
                            const int32_t *eu, const int32_t *ev, int64_t *k4, int64_t *c4) {
  if (oracle_check_csr(n, rp, col)) return -1;
  for (int64_t i = 0; i < cnt; i++) {
    int64_t u = eu[i], v = ev[i];
    if (!adjacent(rp, col, u, v)) return -2;
    int64_t nk = 0, nc = 0;
    for (int64_t w = 0; w < n; w++)
      for (int64_t r = w + 1; r < n; r++) {
        if (w == u || w == v || r == u || r == v) continue;
        int64_t vs[4] = {u, v, w, r};
        int deg[4] = {0, 0, 0, 0}, edges = 0;
        for (int a = 0; a < 4; a++)
          for (int b = 0; b < 4; b++)
            if (a != b && adjacent(rp, col, vs[a], vs[b])) deg[a]++;
        for (int a = 0; a < 4; a++) edges += deg[a];
        edges /= 2;
        int mx = 0;
        for (int a = 0; a < 4; a++) mx = deg[a] > mx ? deg[a] : mx;
        if (edges == 6) nk++;
        if (edges == 4 && mx == 2) nc++;
      }
    k4[i] = nk;
    c4[i] = nc;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Route 3: the per-edge quantities, literally, one edge at a time.          */
/* ------------------------------------------------------------------------ */

/*
 * For each listed edge e = (u, v):
 *   T[i]  = |Tri_e| = |N(u) ∩ N(v)|                                  (Sec. 3)
 *   K4[i] = #{ {w, r} ⊂ Tri_e : (w, r) ∈ E }        (Corollary "cliq": N_TT1)
 *   C4[i] = #{ (w, r) : w ∈ Star_u, r ∈ Star_v, (w, r) ∈ E }
 *                                                    (Corollary "cyc": N_SuSv1)
 * with Star_u = N(u) \ {v} \ N(v) and Star_v = N(v) \ {u} \ N(u).  The
 * C4 count walks N(w) for w on the smaller star side and tests membership in
 * the other side; the set of pairs counted is the same either way.
 */
int oracle_per_edge(int64_t n, const int32_t *rp, const int32_t *col, int64_t cnt,
                    const int32_t *eu, const int32_t *ev, int64_t *T, int64_t *K4, int64_t *C4) {
  (void)n;
  int64_t cap = 0;
  int32_t *tri = NULL, *su = NULL, *sv = NULL;
  for (int64_t i = 0; i < cnt; i++) {
    int64_t u = eu[i], v = ev[i];
    if (u < 0 || v < 0 || u >= n || v >= n || !adjacent(rp, col, u, v)) {
      free(tri); free(su); free(sv);
      return -2;
    }
    int64_t du = rp[u + 1] - rp[u], dv = rp[v + 1] - rp[v];
    int64_t need = du + dv + 1;
    if (need > cap) {
      free(tri); free(su); free(sv);
      cap = need;
      tri = (int32_t *)malloc(sizeof(int32_t) * cap);
      su = (int32_t *)malloc(sizeof(int32_t) * cap);
      sv = (int32_t *)malloc(sizeof(int32_t) * cap);
      if (!tri || !su || !sv) { free(tri); free(su); free(sv); return -3; }
    }
    /* Step 1 by a merge of the two sorted lists. */
    int64_t nt = 0, nu = 0, nv = 0;
    int64_t a = rp[u], b = rp[v];
    while (a < rp[u + 1] || b < rp[v + 1]) {
      int64_t x = a < rp[u + 1] ? col[a] : INT64_MAX;
      int64_t y = b < rp[v + 1] ? col[b] : INT64_MAX;
      if (x == y) { tri[nt++] = (int32_t)x; a++; b++; }
      else if (x < y) { if (x != v) su[nu++] = (int32_t)x; a++; }
      else { if (y != u) sv[nv++] = (int32_t)y; b++; }
    }
    T[i] = nt;
    /* 4-cliques: adjacent pairs inside Tri_e. */
    int64_t k = 0;
    for (int64_t p = 0; p < nt; p++)
      for (int64_t q = p + 1; q < nt; q++) k += adjacent(rp, col, tri[p], tri[q]);
    K4[i] = k;
    /* 4-cycles: edges between Star_u and Star_v. */
    const int32_t *small = nu <= nv ? su : sv, *other = nu <= nv ? sv : su;
    int64_t ns = nu <= nv ? nu : nv, no = nu <= nv ? nv : nu;
    int64_t c = 0;
    for (int64_t p = 0; p < ns; p++) {
      int64_t w = small[p];
      for (int64_t j = rp[w]; j < rp[w + 1]; j++) {
        int64_t r = col[j];
        int64_t lo = 0, hi = no;
        while (lo < hi) {
          int64_t mid = (lo + hi) / 2;
          if (other[mid] < r) lo = mid + 1; else hi = mid;
        }
        if (lo < no && other[lo] == r) c++;
      }
    }
    C4[i] = c;
  }
  free(tri); free(su); free(sv);
  return 0;
}

/* Canonical edge order: (u, v) with u < v, u ascending, then v ascending as
 * in u's list.  Writes m pairs. */
int64_t oracle_edges(int64_t n, const int32_t *rp, const int32_t *col, int32_t *eu, int32_t *ev) {
  int64_t k = 0;
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++)
      if (col[j] > u) {
        if (eu) eu[k] = (int32_t)u;
        if (ev) ev[k] = col[j];
        k++;
      }
  return k;
}

/* ------------------------------------------------------------------------ */
/* Route 2: non-induced pattern counts, inverted.                            */
/* ------------------------------------------------------------------------ */

/*
 * Non-induced counts (copies of a pattern as a subgraph, not necessarily
 * induced) of the connected patterns on 3 and 4 vertices:
 *   P2  2-paths       sum_v C(d_v, 2)
 *   t   triangles
 *   S3  3-stars       sum_v C(d_v, 3)
 *   P3  3-edge paths  sum_{uv in E} (d_u - 1)(d_v - 1) - 3t
 *   C4  4-cycles      (1/2) sum_{a<b} C(c_ab, 2), c_ab = |N(a) ∩ N(b)|
 *   TT  tailed tri.   sum_v t_v (d_v - 2)
 *   D   diamonds      sum_{e in E} C(t_e, 2)
 *   K4  4-cliques
 * Each non-induced count equals sum over induced classes H' of
 * ind(H') * (number of spanning copies of the pattern inside H'):
 *   D  = g4_2 + 6 K4
 *   C4 = g4_4 + g4_2 + 3 K4
 *   TT = g4_3 + 4 g4_2 + 12 K4
 *   S3 = g4_5 + g4_3 + 2 g4_2 + 4 K4
 *   P3 = g4_6 + 2 g4_3 + 4 g4_4 + 6 g4_2 + 12 K4
 * and (pattern, extra vertices) pairs give the disconnected classes:
 *   m (n-2)        = g3_3 + 2 g3_2 + 3 g3_1
 *   t (n-3)        = g4_7 + g4_3 + 2 g4_2 + 4 K4
 *   C(m,2) - P2    = g4_9 + g4_6 + 2 g4_4 + g4_3 + 2 g4_2 + 3 K4
 *   P2 (n-3)       = g4_8 + 3 g4_7 + 2 g4_6 + 3 g4_5 + 4 g4_4 + 5 g4_3
 *                    + 8 g4_2 + 12 K4
 *   m C(n-2, 2)    = g4_10 + 2 (g4_8 + g4_9) + 3 (g4_5 + g4_6 + g4_7)
 *                    + 4 (g4_3 + g4_4) + 5 g4_2 + 6 K4
 * The remaining class of each size is C(n, k) minus the others.
 *
 * Triangles, cliques and 4-cycles are enumerated once each under the order
 * x < y iff (d_x, x) < (d_y, y) (Chiba and Nishizeki), so the route stays
 * usable on graphs with tens of millions of edges.
 */
int oracle_identity_route(int64_t n, const int32_t *rp, const int32_t *col, orc_u128 out[17]) {
  if (oracle_check_csr(n, rp, col)) return -1;
  int64_t m2 = rp[n];
  u128 m = (u128)(m2 / 2);
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (n + 1)); /* vertex -> position in order */
  int64_t *eid = (int64_t *)malloc(sizeof(int64_t) * (m2 + 1)); /* CSR slot -> undirected id */
  int64_t *te = (int64_t *)calloc((size_t)(m2 / 2 + 1), sizeof(int64_t));
  int64_t *tv = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  int64_t *mark2 = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  int64_t *touched = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  if (!deg || !pos || !eid || !te || !tv || !mark || !mark2 || !cnt || !touched || !ord) {
    free(deg); free(pos); free(eid); free(te); free(tv); free(mark); free(mark2); free(cnt);
    free(touched); free(ord);
    return -3;
  }
  for (int64_t v = 0; v < n; v++) deg[v] = rp[v + 1] - rp[v];
  /* Order vertices by (degree, id): counting sort on degree, stable in id. */
  {
    int64_t maxd = 0;
    for (int64_t v = 0; v < n; v++) maxd = deg[v] > maxd ? deg[v] : maxd;
    int64_t *bucket = (int64_t *)calloc((size_t)(maxd + 2), sizeof(int64_t));
    for (int64_t v = 0; v < n; v++) bucket[deg[v] + 1]++;
    for (int64_t d = 0; d <= maxd; d++) bucket[d + 1] += bucket[d];
    for (int64_t v = 0; v < n; v++) { pos[v] = bucket[deg[v]]++; ord[pos[v]] = v; }
    free(bucket);
  }
  /* Undirected edge ids: canonical order (u < v). */
  {
    int64_t k = 0;
    for (int64_t u = 0; u < n; u++)
      for (int64_t j = rp[u]; j < rp[u + 1]; j++)
        if (col[j] > u) eid[j] = k++;
    for (int64_t u = 0; u < n; u++)
      for (int64_t j = rp[u]; j < rp[u + 1]; j++)
        if (col[j] < u) {
          int64_t w = col[j], lo = rp[w], hi = rp[w + 1];
          while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (col[mid] < u) lo = mid + 1; else hi = mid;
          }
          eid[j] = eid[lo];
        }
  }
  /* Upper lists: up[x] = neighbours later than x in the order, each with the
   * undirected id of its edge; every triangle and clique below is listed once
   * from its lowest vertex, reading upper lists only. */
  int64_t *up_ptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
  int64_t *up_col = (int64_t *)malloc(sizeof(int64_t) * (m2 / 2 + 1));
  int64_t *up_eid = (int64_t *)malloc(sizeof(int64_t) * (m2 / 2 + 1));
  if (!up_ptr || !up_col || !up_eid) {
    free(up_ptr); free(up_col); free(up_eid);
    free(deg); free(pos); free(eid); free(te); free(tv); free(mark); free(mark2); free(cnt);
    free(touched); free(ord);
    return -3;
  }
  for (int64_t x = 0; x < n; x++) {
    up_ptr[x + 1] = up_ptr[x];
    for (int64_t j = rp[x]; j < rp[x + 1]; j++)
      if (pos[col[j]] > pos[x]) {
        up_col[up_ptr[x + 1]] = col[j];
        up_eid[up_ptr[x + 1]] = eid[j];
        up_ptr[x + 1]++;
      }
  }
  /* Triangles x < y < z: y in up(x), z in up(y) and in up(x).
   * mark[z] = 1 + undirected id of (x, z). */
  u128 t = 0, k4 = 0;
  for (int64_t v = 0; v < n; v++) { mark[v] = 0; mark2[v] = 0; }
  for (int64_t x = 0; x < n; x++) {
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) mark[up_col[j]] = up_eid[j] + 1;
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) {
      int64_t y = up_col[j];
      for (int64_t q = up_ptr[y]; q < up_ptr[y + 1]; q++) {
        int64_t z = up_col[q];
        if (!mark[z]) continue;
        t++;
        te[up_eid[j]]++;
        te[up_eid[q]]++;
        te[mark[z] - 1]++;
        tv[x]++; tv[y]++; tv[z]++;
      }
    }
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) mark[up_col[j]] = 0;
  }
  /* 4-cliques x < y < z < w: y in up(x); z, w in up(x) and up(y); w in up(z). */
  for (int64_t x = 0; x < n; x++) {
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) mark[up_col[j]] = 1;
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) {
      int64_t y = up_col[j];
      for (int64_t q = up_ptr[y]; q < up_ptr[y + 1]; q++)
        if (mark[up_col[q]]) mark2[up_col[q]] = 1;
      for (int64_t q = up_ptr[y]; q < up_ptr[y + 1]; q++) {
        int64_t z = up_col[q];
        if (!mark2[z]) continue;
        for (int64_t r = up_ptr[z]; r < up_ptr[z + 1]; r++)
          if (mark2[up_col[r]]) k4++;
      }
      for (int64_t q = up_ptr[y]; q < up_ptr[y + 1]; q++) mark2[up_col[q]] = 0;
    }
    for (int64_t j = up_ptr[x]; j < up_ptr[x + 1]; j++) mark[up_col[j]] = 0;
  }
  free(up_ptr); free(up_col); free(up_eid);
  /* 4-cycles (non-induced): each cycle has one highest vertex x; with y the
   * vertex opposite x, the cycle is two paths x - v - y with v, y below x.
   * cnt[y] counts such paths; the cycles with that (x, y) are C(cnt[y], 2). */
  u128 c4 = 0;
  for (int64_t x = 0; x < n; x++) {
    int64_t nt = 0;
    for (int64_t j = rp[x]; j < rp[x + 1]; j++) {
      int64_t v = col[j];
      if (pos[v] >= pos[x]) continue;
      for (int64_t q = rp[v]; q < rp[v + 1]; q++) {
        int64_t y = col[q];
        if (pos[y] >= pos[x]) continue;
        if (cnt[y]++ == 0) touched[nt++] = y;
      }
    }
    for (int64_t i = 0; i < nt; i++) {
      c4 += choose((u128)cnt[touched[i]], 2);
      cnt[touched[i]] = 0;
    }
  }
  u128 P2 = 0, S3 = 0, P3 = 0, TT = 0, D = 0;
  for (int64_t v = 0; v < n; v++) {
    P2 += choose((u128)deg[v], 2);
    S3 += choose((u128)deg[v], 3);
    if (deg[v] >= 2) TT += (u128)tv[v] * (u128)(deg[v] - 2);
  }
  for (int64_t u = 0; u < n; u++)
    for (int64_t j = rp[u]; j < rp[u + 1]; j++)
      if (col[j] > u) {
        int64_t v = col[j];
        P3 += (u128)(deg[u] - 1) * (u128)(deg[v] - 1);
        D += choose((u128)te[eid[j]], 2);
      }
  P3 -= 3 * t;

  i128 g[17];
  u128 N = (u128)n;
  g[0] = (i128)m;
  g[1] = (i128)choose(N, 2) - (i128)m;
  g[2] = (i128)t;
  g[3] = (i128)P2 - 3 * (i128)t;
  g[4] = (n >= 2 ? (i128)m * (i128)(N - 2) : 0) - 2 * g[3] - 3 * g[2];
  g[5] = (i128)choose(N, 3) - g[2] - g[3] - g[4];
  i128 K = (i128)k4;
  g[6] = K;
  g[7] = (i128)D - 6 * K;
  g[9] = (i128)c4 - g[7] - 3 * K;
  g[8] = (i128)TT - 4 * g[7] - 12 * K;
  g[10] = (i128)S3 - g[8] - 2 * g[7] - 4 * K;
  g[11] = (i128)P3 - 2 * g[8] - 4 * g[9] - 6 * g[7] - 12 * K;
  i128 n3 = n >= 3 ? (i128)(N - 3) : 0;
  g[12] = (i128)t * n3 - g[8] - 2 * g[7] - 4 * K;
  g[14] = (i128)choose(m, 2) - (i128)P2 - g[11] - 2 * g[9] - g[8] - 2 * g[7] - 3 * K;
  g[13] = (i128)P2 * n3 - 3 * g[12] - 2 * g[11] - 3 * g[10] - 4 * g[9] - 5 * g[8] - 8 * g[7] -
          12 * K;
  g[15] = (n >= 2 ? (i128)m * (i128)choose(N - 2, 2) : 0) - 2 * (g[13] + g[14]) -
          3 * (g[10] + g[11] + g[12]) - 4 * (g[8] + g[9]) - 5 * g[7] - 6 * K;
  i128 s = 0;
  for (int i = 6; i <= 15; i++) s += g[i];
  g[16] = (i128)choose(N, 4) - s;

  free(deg); free(pos); free(eid); free(te); free(tv); free(mark); free(mark2); free(cnt);
  free(touched); free(ord);
  for (int i = 0; i < 17; i++)
    if (g[i] < 0) return -5;
  for (int i = 0; i < 17; i++) put(&out[i], (u128)g[i]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-edge local 4-node vectors (edge orbits).                             */
/* ------------------------------------------------------------------------ */
/*
 * For an edge e = (u, v), every other vertex w has a type relative to e
 * (Section 4.2): T (adjacent to u and v, w in Tri_e), Su (adjacent to u
 * only), Sv (adjacent to v only) or I (adjacent to neither).  The 4-subsets
 * containing e are the pairs {w, r}; their induced graphlet is fixed by the
 * two types and by whether w and r are adjacent.  The paper writes N_{a,b}
 * for the number of pairs of types (a, b), and N_{a,b,1} / N_{a,b,0} for
 * those whose two vertices are / are not adjacent.
 *
 * Output per edge, 17 int64 values (the graphlet and e's place in it):
 *   [0] |Tri_e|          triangle                            (g3_1)
 *   [1] |Su| + |Sv|      2-star                              (g3_2)
 *   [2] I_e              3-node-1-edge                       (g3_3)
 *   [3] N_{T,T,1}        4-clique                            (g4_1)
 *   [4] N_{T,T,0}        chordal cycle, e the chord          (g4_2)
 *   [5] N_{T,S,1}        chordal cycle, e on the cycle       (g4_2)
 *   [6] N_{T,S,0}        tailed triangle, e in the triangle at the tail's vertex (g4_3)
 *   [7] N_{T,I,1}        tailed triangle, e in the triangle away from the tail  (g4_3)
 *   [8] N_{S,S,1}        tailed triangle, e the tail         (g4_3)
 *   [9] N_{Su,Sv,1}      4-cycle                             (g4_4)
 *  [10] N_{S,S,0}        3-star                              (g4_5)
 *  [11] N_{Su,Sv,0}      4-path, e in the middle             (g4_6)
 *  [12] N_{S,I,1}        4-path, e at an end                 (g4_6)
 *  [13] N_{T,I,0}        4-node-1-triangle                   (g4_7)
 *  [14] N_{S,I,0}        4-node-2-star                       (g4_8)
 *  [15] N_{I,I,1}        4-node-2-edge                       (g4_9)
 *  [16] N_{I,I,0}        4-node-1-edge                       (g4_10)
 * where S,S pairs two vertices of the same star (Su,Su or Sv,Sv), T,S a T
 * vertex with a star vertex, and S,I a star vertex with an I vertex.
 */
#define ORC_LOCAL 17

enum { TY_T = 0, TY_SU = 1, TY_SV = 2, TY_I = 3, TY_UV = 4 };

/* The types route: unrestricted counts from the type sizes (Section 4.2),
 * restricted "1" counts by looking at every edge (w, r) of the graph. */
int oracle_edge_local(int64_t n, const int32_t *rp, const int32_t *col, int64_t cnt,
                      const int32_t *eu, const int32_t *ev, int64_t *out) {
  unsigned char *ty = (unsigned char *)malloc(n > 0 ? (size_t)n : 1);
  if (!ty) return -3;
  for (int64_t i = 0; i < cnt; i++) {
    const int64_t u = eu[i], v = ev[i];
    if (u < 0 || v < 0 || u >= n || v >= n || !adjacent(rp, col, u, v)) {
      free(ty);
      return -2;
    }
    for (int64_t w = 0; w < n; w++) {
      const int au = adjacent(rp, col, w, u), av = adjacent(rp, col, w, v);
      ty[w] = au && av ? TY_T : au ? TY_SU : av ? TY_SV : TY_I;
    }
    ty[u] = ty[v] = TY_UV;
    int64_t sz[4] = {0, 0, 0, 0};
    for (int64_t w = 0; w < n; w++)
      if (ty[w] != TY_UV) sz[ty[w]]++;
    /* adjacent pairs by type pair: one[a][b], a <= b */
    int64_t one[4][4];
    memset(one, 0, sizeof one);
    for (int64_t w = 0; w < n; w++) {
      if (ty[w] == TY_UV) continue;
      for (int64_t j = rp[w]; j < rp[w + 1]; j++) {
        const int64_t r = col[j];
        if (r <= w || ty[r] == TY_UV) continue;
        int a = ty[w], b = ty[r];
        if (a > b) { int t = a; a = b; b = t; }
        one[a][b]++;
      }
    }
    const int64_t T = sz[TY_T], Su = sz[TY_SU], Sv = sz[TY_SV], I = sz[TY_I];
    const int64_t nTT = T * (T - 1) / 2, nTS = T * (Su + Sv);
    const int64_t nSS = Su * (Su - 1) / 2 + Sv * (Sv - 1) / 2, nSuSv = Su * Sv;
    const int64_t nTI = T * I, nSI = (Su + Sv) * I, nII = I * (I - 1) / 2;
    const int64_t oTT = one[TY_T][TY_T], oTS = one[TY_T][TY_SU] + one[TY_T][TY_SV];
    const int64_t oSS = one[TY_SU][TY_SU] + one[TY_SV][TY_SV], oSuSv = one[TY_SU][TY_SV];
    const int64_t oTI = one[TY_T][TY_I], oSI = one[TY_SU][TY_I] + one[TY_SV][TY_I];
    const int64_t oII = one[TY_I][TY_I];
    int64_t *o = out + i * ORC_LOCAL;
    o[0] = T;
    o[1] = Su + Sv;
    o[2] = I;
    o[3] = oTT;
    o[4] = nTT - oTT;
    o[5] = oTS;
    o[6] = nTS - oTS;
    o[7] = oTI;
    o[8] = oSS;
    o[9] = oSuSv;
    o[10] = nSS - oSS;
    o[11] = nSuSv - oSuSv;
    o[12] = oSI;
    o[13] = nTI - oTI;
    o[14] = nSI - oSI;
    o[15] = oII;
    o[16] = nII - oII;
  }
  free(ty);
  return 0;
}

/* The definition route: every 3- and 4-subset containing u and v is
 * classified by Table 1 (oracle_classify4), and e's place in its graphlet
 * is read from the degrees of u and v inside the subset. */
int oracle_edge_local_brute(int64_t n, const int32_t *rp, const int32_t *col, int64_t cnt,
                            const int32_t *eu, const int32_t *ev, int64_t *out) {
  for (int64_t i = 0; i < cnt; i++) {
    const int64_t u = eu[i], v = ev[i];
    if (u < 0 || v < 0 || u >= n || v >= n || !adjacent(rp, col, u, v)) return -2;
    int64_t *o = out + i * ORC_LOCAL;
    memset(o, 0, sizeof(int64_t) * ORC_LOCAL);
    for (int64_t w = 0; w < n; w++) {
      if (w == u || w == v) continue;
      const int e3 = 1 + adjacent(rp, col, u, w) + adjacent(rp, col, v, w);
      o[3 - e3]++; /* 3 edges: triangle, 2: 2-star, 1: one edge */
    }
    for (int64_t w = 0; w < n; w++)
      for (int64_t r = w + 1; r < n; r++) {
        if (w == u || w == v || r == u || r == v) continue;
        const int64_t vs[4] = {u, v, w, r};
        int deg[4] = {0, 0, 0, 0}, A[4][4];
        for (int a = 0; a < 4; a++)
          for (int b = 0; b < 4; b++) {
            A[a][b] = a != b && adjacent(rp, col, vs[a], vs[b]);
            deg[a] += A[a][b];
          }
        int edges = 0, mx = 0;
        for (int a = 0; a < 4; a++) {
          edges += deg[a];
          mx = deg[a] > mx ? deg[a] : mx;
        }
        edges /= 2;
        const int g = oracle_classify4(edges, mx, components(4, A));
        const int du = deg[0], dv = deg[1];
        const int lo = du < dv ? du : dv, hi = du < dv ? dv : du;
        switch (g) { /* Table 1 row index: 0 = g4_1 ... 9 = g4_10 */
          case 0: o[3]++; break;                               /* 4-clique */
          case 1: o[lo == 3 ? 4 : 5]++; break;                 /* chordal cycle */
          case 2: o[lo == 1 ? 8 : (hi == 3 ? 6 : 7)]++; break; /* tailed triangle */
          case 3: o[9]++; break;                               /* 4-cycle */
          case 4: o[10]++; break;                              /* 3-star */
          case 5: o[lo == 2 ? 11 : 12]++; break;               /* 4-path */
          case 6: o[13]++; break;                              /* 4-node-1-triangle */
          case 7: o[14]++; break;                              /* 4-node-2-star */
          case 8: o[15]++; break;                              /* 4-node-2-edge */
          case 9: o[16]++; break;                              /* 4-node-1-edge */
          default: return -4; /* e is an edge: never independent */
        }
      }
  }
  return 0;
}
