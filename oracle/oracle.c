/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for triangle
 * counting, per-edge support, k-truss and truss decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything here is integer and exact.  Each function names the passage of
 * the paper (Samsi et al., "Static Graph Challenge: Subgraph Isomorphism",
 * 2017) whose definition it writes out.
 *
 * Conventions
 *   - Vertex ids are int32 in [0, n).  (The paper's files number vertices
 *     1..n, Sec. II; `one_based` subtracts 1.)
 *   - A canonical edge list is the set E = {{u, v}} of an undirected simple
 *     graph written as pairs u < v in lexicographic order; the position of a
 *     pair is its edge id, i.e. the row of the incidence matrix E (Sec. III-B).
 *     Every per-edge output (support, truss membership, truss number) is
 *     indexed by that id.
 *   - Counts are int64; supports and truss numbers are int32.
 *   - Single thread, as the paper's serial implementations; the one
 *     exception is oracle_triangle_count_threads, the same count with the
 *     outer loop split over threads (for timing the oracle on every host
 *     core; its result is tested equal to the serial one).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Normalisation (Sec. II: integer ids, loops removed, directed graphs made   */
/* undirected).  Output is the canonical edge list; duplicates collapse.      */
/* ------------------------------------------------------------------------- */

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

/* Returns m (>= 0), -1 if an id falls outside [0, n), -2 on allocation failure.
 * u_out / v_out must hold n_pairs entries. */
int64_t oracle_normalise(const int32_t *src, const int32_t *dst, int64_t n_pairs,
                         int32_t n, int32_t one_based, int32_t *u_out,
                         int32_t *v_out) {
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_pairs + 1));
  if (!key) return -2;
  int64_t k = 0;
  for (int64_t i = 0; i < n_pairs; ++i) {
    int64_t a = (int64_t)src[i] - (one_based ? 1 : 0);
    int64_t b = (int64_t)dst[i] - (one_based ? 1 : 0);
    if (a < 0 || a >= n || b < 0 || b >= n) { free(key); return -1; }
    if (a == b) continue;                        /* self-loop: dropped */
    uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
    key[k++] = (lo << 32) | hi;                  /* undirected: {min, max} */
  }
  qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t m = 0;
  for (int64_t i = 0; i < k; ++i) {
    if (i > 0 && key[i] == key[i - 1]) continue; /* duplicate pair */
    u_out[m] = (int32_t)(key[i] >> 32);
    v_out[m] = (int32_t)(key[i] & 0xFFFFFFFFu);
    ++m;
  }
  free(key);
  return m;
}

/* ------------------------------------------------------------------------- */
/* Undirected adjacency with edge ids: for each vertex x, the sorted list of   */
/* neighbours y and the id of edge {x, y}.  This is the row x of A (and the    */
/* column structure of E), Sec. III.                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t n;
  int64_t m;
  int64_t *off;   /* n + 1 */
  int32_t *nbr;   /* 2m */
  int32_t *eid;   /* 2m */
} adj_t;

static void adj_free(adj_t *g) {
  free(g->off); free(g->nbr); free(g->eid);
  g->off = NULL; g->nbr = NULL; g->eid = NULL;
}

typedef struct { int32_t y, e; } ye_t;
static int cmp_ye(const void *a, const void *b) {
  int32_t x = ((const ye_t *)a)->y, y = ((const ye_t *)b)->y;
  return (x > y) - (x < y);
}

static int adj_build(adj_t *g, int32_t n, int64_t m, const int32_t *u,
                     const int32_t *v) {
  g->n = n; g->m = m;
  g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  g->eid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  ye_t *tmp = NULL;
  if (!g->off || !g->nbr || !g->eid || !fill) { free(fill); adj_free(g); return -1; }
  for (int64_t e = 0; e < m; ++e) { g->off[u[e] + 1]++; g->off[v[e] + 1]++; }
  for (int32_t x = 0; x < n; ++x) g->off[x + 1] += g->off[x];
  memcpy(fill, g->off, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < m; ++e) {
    g->nbr[fill[u[e]]] = v[e]; g->eid[fill[u[e]]++] = (int32_t)e;
    g->nbr[fill[v[e]]] = u[e]; g->eid[fill[v[e]]++] = (int32_t)e;
  }
  free(fill);
  /* sort every list by neighbour id */
  int64_t maxd = 0;
  for (int32_t x = 0; x < n; ++x)
    if (g->off[x + 1] - g->off[x] > maxd) maxd = g->off[x + 1] - g->off[x];
  tmp = (ye_t *)malloc(sizeof(ye_t) * (size_t)(maxd + 1));
  if (!tmp) { adj_free(g); return -1; }
  for (int32_t x = 0; x < n; ++x) {
    int64_t b = g->off[x], d = g->off[x + 1] - b;
    for (int64_t i = 0; i < d; ++i) { tmp[i].y = g->nbr[b + i]; tmp[i].e = g->eid[b + i]; }
    qsort(tmp, (size_t)d, sizeof(ye_t), cmp_ye);
    for (int64_t i = 0; i < d; ++i) { g->nbr[b + i] = tmp[i].y; g->eid[b + i] = tmp[i].e; }
  }
  free(tmp);
  return 0;
}

/* Position of y in the sorted range nbr[lo, hi), or -1. */
static int64_t find_sorted(const int32_t *nbr, int64_t lo, int64_t hi, int32_t y) {
  const int64_t end = hi;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (nbr[mid] < y) lo = mid + 1;
    else hi = mid;
  }
  return (lo < end && nbr[lo] == y) ? lo : -1;
}

/* ------------------------------------------------------------------------- */
/* Triangle count (Sec. III-A: a triangle is a set of three mutually adjacent  */
/* vertices).  Forward listing: orient each edge from the lower to the higher  */
/* vertex of the strict total order  x < y  iff  (deg x, -x) < (deg y, -y),    */
/* so each triangle appears exactly once as a pair of out-edges x->y, x->z     */
/* with y->z (the masked product sum(A .* (L L)) of Alg. 3, with L taken in    */
/* this order).  Intersections are two-pointer merges of sorted lists.         */
/* ------------------------------------------------------------------------- */
static int precedes(const int64_t *deg, int32_t x, int32_t y) {
  if (deg[x] != deg[y]) return deg[x] < deg[y];
  return x > y;
}

int64_t oracle_triangle_count(int32_t n, int64_t m, const int32_t *u,
                              const int32_t *v) {
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t *ooff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  if (!deg || !ooff || !out) { free(deg); free(ooff); free(out); adj_free(&g); return -2; }
  for (int32_t x = 0; x < n; ++x) deg[x] = g.off[x + 1] - g.off[x];
  /* out-lists N+(x): neighbours that x precedes, kept in id order */
  for (int32_t x = 0; x < n; ++x) {
    ooff[x + 1] = ooff[x];
    for (int64_t i = g.off[x]; i < g.off[x + 1]; ++i)
      if (precedes(deg, x, g.nbr[i])) out[ooff[x + 1]++] = g.nbr[i];
  }
  int64_t T = 0;
  for (int32_t x = 0; x < n; ++x) {
    for (int64_t i = ooff[x]; i < ooff[x + 1]; ++i) {
      int32_t y = out[i];
      int64_t a = ooff[x], ae = ooff[x + 1], b = ooff[y], be = ooff[y + 1];
      while (a < ae && b < be) {                 /* |N+(x) cap N+(y)| */
        if (out[a] < out[b]) ++a;
        else if (out[a] > out[b]) ++b;
        else { ++T; ++a; ++b; }
      }
    }
  }
  free(deg); free(ooff); free(out); adj_free(&g);
  return T;
}

/* The same count with the vertices x dealt to `nthreads` threads in turn     */
/* (x = t, t + nthreads, ...: a static schedule that spreads the high-degree  */
/* vertices), each thread summing into its own int64 partial.                 */
typedef struct {
  const int64_t *ooff;
  const int32_t *out;
  int32_t n, t, nthreads;
  int64_t partial;
} tc_share_t;

static void *tc_share(void *arg) {
  tc_share_t *w = (tc_share_t *)arg;
  int64_t T = 0;
  for (int32_t x = w->t; x < w->n; x += w->nthreads) {
    for (int64_t i = w->ooff[x]; i < w->ooff[x + 1]; ++i) {
      int32_t y = w->out[i];
      int64_t a = w->ooff[x], ae = w->ooff[x + 1], b = w->ooff[y], be = w->ooff[y + 1];
      while (a < ae && b < be) {
        if (w->out[a] < w->out[b]) ++a;
        else if (w->out[a] > w->out[b]) ++b;
        else { ++T; ++a; ++b; }
      }
    }
  }
  w->partial = T;
  return NULL;
}

int64_t oracle_triangle_count_threads(int32_t n, int64_t m, const int32_t *u,
                                      const int32_t *v, int32_t nthreads) {
  if (nthreads < 1 || nthreads > 1024) return -1;
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t *ooff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  tc_share_t *w = (tc_share_t *)calloc((size_t)nthreads, sizeof(tc_share_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  uint8_t *started = (uint8_t *)calloc((size_t)nthreads, 1);
  if (!deg || !ooff || !out || !w || !th || !started) {
    free(deg); free(ooff); free(out); free(w); free(th); free(started); adj_free(&g);
    return -2;
  }
  for (int32_t x = 0; x < n; ++x) deg[x] = g.off[x + 1] - g.off[x];
  for (int32_t x = 0; x < n; ++x) {
    ooff[x + 1] = ooff[x];
    for (int64_t i = g.off[x]; i < g.off[x + 1]; ++i)
      if (precedes(deg, x, g.nbr[i])) out[ooff[x + 1]++] = g.nbr[i];
  }
  int64_t T = 0;
  for (int32_t t = 0; t < nthreads; ++t) {
    w[t].ooff = ooff; w[t].out = out; w[t].n = n; w[t].t = t; w[t].nthreads = nthreads;
    if (pthread_create(&th[t], NULL, tc_share, &w[t]) == 0) started[t] = 1;
    else tc_share(&w[t]);                        /* no thread: this one does it */
  }
  for (int32_t t = 0; t < nthreads; ++t) {
    if (started[t]) pthread_join(th[t], NULL);
    T += w[t].partial;
  }
  free(deg); free(ooff); free(out); free(w); free(th); free(started); adj_free(&g);
  return T;
}

/* ------------------------------------------------------------------------- */
/* Per-edge support (Sec. III-B): summing the rows of A of the two endpoints   */
/* of edge e gives 2 exactly at their common neighbours, so                    */
/*   s(e) = |N(u) cap N(v)|  =  (A^2 .* A)(u, v)  (the matrix C of Alg. 2).    */
/* Each edge is intersected directly: the smaller list is searched in the      */
/* larger one.                                                                 */
/* ------------------------------------------------------------------------- */
static int32_t common_neighbours(const adj_t *g, int32_t a, int32_t b,
                                 const uint8_t *alive) {
  int64_t la = g->off[a], ha = g->off[a + 1], lb = g->off[b], hb = g->off[b + 1];
  if (ha - la > hb - lb) {                       /* iterate the shorter list */
    int64_t t;
    int32_t tv = a; a = b; b = tv;
    t = la; la = lb; lb = t; t = ha; ha = hb; hb = t;
  }
  int32_t s = 0;
  for (int64_t i = la; i < ha; ++i) {
    if (alive && !alive[g->eid[i]]) continue;    /* edge {a, w} must be alive */
    int64_t j = find_sorted(g->nbr, lb, hb, g->nbr[i]);
    if (j < 0) continue;
    if (alive && !alive[g->eid[j]]) continue;    /* edge {b, w} must be alive */
    ++s;
  }
  return s;
}

int oracle_support(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                   int32_t *s) {
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  for (int64_t e = 0; e < m; ++e) s[e] = common_neighbours(&g, u[e], v[e], NULL);
  adj_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* k-truss, Alg. 4 semantics (Sec. III-B): the k-truss is the subgraph in      */
/* which every edge lies in at least k-2 triangles of the same subgraph.       */
/* Rounds: compute the support of every remaining edge within the remaining    */
/* edges, find every edge with support < k-2, drop them all together, repeat   */
/* until no edge is dropped.  Support is recomputed from scratch each round    */
/* (Alg. 4's incremental update of EA gives the same values).                  */
/* in_out: on entry the edges to start from (1 = present); on exit the k-truss.*/
/* Returns the number of rounds that removed at least one edge, or < 0.        */
/* ------------------------------------------------------------------------- */
int32_t oracle_ktruss_bulk(int32_t n, int64_t m, const int32_t *u,
                           const int32_t *v, int32_t k, uint8_t *in_out) {
  if (k < 2) return -1;
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  if (!s) { adj_free(&g); return -2; }
  int32_t rounds = 0;
  for (;;) {
    for (int64_t e = 0; e < m; ++e)
      s[e] = in_out[e] ? common_neighbours(&g, u[e], v[e], in_out) : 0;
    int64_t dropped = 0;
    for (int64_t e = 0; e < m; ++e)
      if (in_out[e] && s[e] < k - 2) { in_out[e] = 0; ++dropped; }
    if (dropped == 0) break;
    ++rounds;
  }
  free(s); adj_free(&g);
  return rounds;
}

/* ------------------------------------------------------------------------- */
/* Support by triangle listing (an independent second route to the same       */
/* numbers): list every triangle once by forward listing in the order of      */
/* oracle_triangle_count, and add one to each of its three edges.  The         */
/* listing also yields, per edge, the ids of the other two edges of each of    */
/* its triangles (the "triangle index" used by peeling below).                 */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t m;
  int64_t *off;   /* m + 1: triangles of edge e are pair[off[e] .. off[e+1]) */
  int32_t *pair;  /* 2 * 3T: the other two edge ids of each triangle of e   */
} tri_index_t;

static void tri_index_free(tri_index_t *t) {
  free(t->off); free(t->pair);
  t->off = NULL; t->pair = NULL;
}

/* Forward listing over oriented lists that carry edge ids.  If cnt != NULL,
 * add 1 to cnt[e] for each edge of each triangle; if t != NULL, append the
 * other two edge ids at fill[e].  Returns T. */
static int64_t list_triangles(const adj_t *g, int64_t *cnt, tri_index_t *t, int64_t *fill) {
  const int32_t n = g->n;
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t *ooff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *out = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->m + 1));
  int32_t *oid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(g->m + 1));
  if (!deg || !ooff || !out || !oid) { free(deg); free(ooff); free(out); free(oid); return -2; }
  for (int32_t x = 0; x < n; ++x) deg[x] = g->off[x + 1] - g->off[x];
  for (int32_t x = 0; x < n; ++x) {
    ooff[x + 1] = ooff[x];
    for (int64_t i = g->off[x]; i < g->off[x + 1]; ++i)
      if (precedes(deg, x, g->nbr[i])) {
        out[ooff[x + 1]] = g->nbr[i];
        oid[ooff[x + 1]++] = g->eid[i];
      }
  }
  int64_t T = 0;
  for (int32_t x = 0; x < n; ++x) {
    for (int64_t i = ooff[x]; i < ooff[x + 1]; ++i) {
      const int32_t y = out[i];
      const int32_t exy = oid[i];
      int64_t a = ooff[x], ae = ooff[x + 1], b = ooff[y], be = ooff[y + 1];
      while (a < ae && b < be) {
        if (out[a] < out[b]) ++a;
        else if (out[a] > out[b]) ++b;
        else {                          /* triangle {x, y, z}, z = out[a] */
          const int32_t exz = oid[a], eyz = oid[b];
          ++T;
          if (cnt) { cnt[exy]++; cnt[exz]++; cnt[eyz]++; }
          if (t) {
            int64_t q;
            q = fill[exy]++; t->pair[2 * q] = exz; t->pair[2 * q + 1] = eyz;
            q = fill[exz]++; t->pair[2 * q] = exy; t->pair[2 * q + 1] = eyz;
            q = fill[eyz]++; t->pair[2 * q] = exy; t->pair[2 * q + 1] = exz;
          }
          ++a; ++b;
        }
      }
    }
  }
  free(deg); free(ooff); free(out); free(oid);
  return T;
}

int oracle_support_listing(int32_t n, int64_t m, const int32_t *u, const int32_t *v,
                           int32_t *s) {
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  int64_t *cnt = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
  if (!cnt) { adj_free(&g); return -2; }
  int64_t T = list_triangles(&g, cnt, NULL, NULL);
  for (int64_t e = 0; e < m; ++e) s[e] = (int32_t)cnt[e];
  free(cnt); adj_free(&g);
  return T < 0 ? -2 : 0;
}

static int tri_index_build(const adj_t *g, tri_index_t *t) {
  const int64_t m = g->m;
  t->m = m;
  t->off = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  if (!t->off || !fill) { free(fill); free(t->off); t->off = NULL; return -2; }
  if (list_triangles(g, t->off + 1, NULL, NULL) < 0) { free(fill); return -2; }
  for (int64_t e = 0; e < m; ++e) t->off[e + 1] += t->off[e];   /* prefix sums */
  t->pair = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * t->off[m] + 2));
  if (!t->pair) { free(fill); return -2; }
  memcpy(fill, t->off, sizeof(int64_t) * (size_t)m);
  list_triangles(g, NULL, t, fill);
  free(fill);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* k-truss by one-edge-at-a-time peeling (an independent second algorithm, in  */
/* the style of the truss work the paper cites in Sec. III-B): start from the  */
/* support of every present edge, queue every edge below k-2, and on removing  */
/* edge e decrement the other two edges of every triangle of e whose three     */
/* edges are all still present (each destroyed triangle is counted once: it    */
/* is destroyed by whichever of its edges is removed first).                   */
/* in_out as for oracle_ktruss_bulk.  Returns 0 or < 0.                        */
/* ------------------------------------------------------------------------- */
static void peel_edge(const tri_index_t *t, int64_t e, uint8_t *alive, int32_t *s,
                      int32_t thr, uint8_t *queued, int64_t *queue, int64_t *qtail) {
  alive[e] = 0;
  for (int64_t q = t->off[e]; q < t->off[e + 1]; ++q) {
    const int32_t e1 = t->pair[2 * q], e2 = t->pair[2 * q + 1];
    if (!alive[e1] || !alive[e2]) continue;     /* already destroyed */
    if (--s[e1] < thr && !queued[e1]) { queued[e1] = 1; queue[(*qtail)++] = e1; }
    if (--s[e2] < thr && !queued[e2]) { queued[e2] = 1; queue[(*qtail)++] = e2; }
  }
}

/* support of every present edge within the present edges, from the index */
static void present_support(const tri_index_t *t, const uint8_t *alive, int32_t *s) {
  for (int64_t e = 0; e < t->m; ++e) {
    int32_t c = 0;
    if (alive[e])
      for (int64_t q = t->off[e]; q < t->off[e + 1]; ++q)
        c += alive[t->pair[2 * q]] && alive[t->pair[2 * q + 1]];
    s[e] = c;
  }
}

int32_t oracle_ktruss_peel(int32_t n, int64_t m, const int32_t *u,
                           const int32_t *v, int32_t k, uint8_t *in_out) {
  if (k < 2) return -1;
  adj_t g;
  tri_index_t t = {0, NULL, NULL};
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  if (tri_index_build(&g, &t) != 0) { tri_index_free(&t); adj_free(&g); return -2; }
  adj_free(&g);
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  uint8_t *queued = (uint8_t *)calloc((size_t)m + 1, 1);
  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
  if (!s || !queued || !queue) { free(s); free(queued); free(queue); tri_index_free(&t); return -2; }
  int64_t qh = 0, qt = 0;
  present_support(&t, in_out, s);
  for (int64_t e = 0; e < m; ++e)
    if (in_out[e] && s[e] < k - 2) { queued[e] = 1; queue[qt++] = e; }
  while (qh < qt) peel_edge(&t, queue[qh++], in_out, s, k - 2, queued, queue, &qt);
  free(s); free(queued); free(queue); tri_index_free(&t);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Peeling without a triangle index (a third route, for graphs whose index of  */
/* 3T edge pairs does not fit in memory).  The same one-edge-at-a-time rule as */
/* peel_edge: on removing edge {a, b}, every triangle {a, b, w} whose edges    */
/* {a, w} and {b, w} are both still present is destroyed once, and those two   */
/* edges lose 1.  The triangles are found by intersecting the adjacency lists  */
/* of a and b directly: the shorter list is walked in increasing order and     */
/* each neighbour w is binary-searched in the other list, from where the       */
/* previous search ended (the walked ids only grow).  Entries of removed edges */
/* stay in a list until they are more than half of it; the list is then        */
/* rewritten, in order, without them.  Memory is O(n + m).                      */
/* ------------------------------------------------------------------------- */
typedef struct {
  adj_t g;          /* list x occupies g.nbr / g.eid [g.off[x], g.off[x] + len[x]) */
  int64_t *len;     /* n: entries still stored in list x */
  int64_t *ndead;   /* n: stored entries of list x whose edge has been removed */
} live_lists_t;

static void live_lists_free(live_lists_t *L) {
  adj_free(&L->g); free(L->len); free(L->ndead);
  L->len = NULL; L->ndead = NULL;
}

/* list x without the entries of removed edges, order kept */
static void drop_removed(live_lists_t *L, int32_t x, const uint8_t *alive) {
  const int64_t b = L->g.off[x], e = b + L->len[x];
  int64_t w = b;
  for (int64_t i = b; i < e; ++i)
    if (alive[L->g.eid[i]]) { L->g.nbr[w] = L->g.nbr[i]; L->g.eid[w] = L->g.eid[i]; ++w; }
  L->len[x] = w - b;
  L->ndead[x] = 0;
}

/* adjacency of the present edges (alive[e] = 1) */
static int live_lists_build(live_lists_t *L, int32_t n, int64_t m, const int32_t *u,
                            const int32_t *v, const uint8_t *alive) {
  L->len = NULL; L->ndead = NULL;
  if (adj_build(&L->g, n, m, u, v) != 0) return -2;
  L->len = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  L->ndead = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!L->len || !L->ndead) { live_lists_free(L); return -2; }
  for (int32_t x = 0; x < n; ++x) {
    L->len[x] = L->g.off[x + 1] - L->g.off[x];
    drop_removed(L, x, alive);
  }
  return 0;
}

static void lose_one(int32_t *s, int32_t e, int32_t thr, uint8_t *queued, int64_t *queue,
                     int64_t *qtail) {
  s[e] -= 1;
  if (s[e] < thr && !queued[e]) { queued[e] = 1; queue[(*qtail)++] = e; }
}

static void peel_edge_by_search(live_lists_t *L, const int32_t *u, const int32_t *v,
                                int64_t e, uint8_t *alive, int32_t *s, int32_t thr,
                                uint8_t *queued, int64_t *queue, int64_t *qtail) {
  int32_t a = u[e], b = v[e];
  alive[e] = 0;
  if (L->len[a] > L->len[b]) { int32_t t = a; a = b; b = t; }   /* walk the shorter */
  const int32_t *nbr = L->g.nbr, *eid = L->g.eid;
  const int64_t ia = L->g.off[a], ea = ia + L->len[a];
  const int64_t hb = L->g.off[b] + L->len[b];
  int64_t lb = L->g.off[b];
  for (int64_t i = ia; i < ea; ++i) {
    const int32_t eaw = eid[i];
    if (!alive[eaw]) continue;                    /* {a, w} already removed */
    const int32_t w = nbr[i];
    int64_t lo = lb, hi = hb;                     /* first entry of b's list >= w */
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (nbr[mid] < w) lo = mid + 1;
      else hi = mid;
    }
    lb = lo;
    if (lo == hb || nbr[lo] != w) continue;       /* w is not a neighbour of b */
    const int32_t ebw = eid[lo];
    if (!alive[ebw]) continue;                    /* {b, w} removed: destroyed before */
    lose_one(s, eaw, thr, queued, queue, qtail);
    lose_one(s, ebw, thr, queued, queue, qtail);
  }
  L->ndead[a] += 1;
  L->ndead[b] += 1;
  if (2 * L->ndead[a] > L->len[a]) drop_removed(L, a, alive);
  if (2 * L->ndead[b] > L->len[b]) drop_removed(L, b, alive);
}

/* k-truss by peeling without a triangle index; in_out as for oracle_ktruss_bulk.
 * The support of each present edge within the present edges is counted by
 * the plain definition before peeling starts.  Returns 0 or < 0. */
int32_t oracle_ktruss_search(int32_t n, int64_t m, const int32_t *u,
                             const int32_t *v, int32_t k, uint8_t *in_out) {
  if (k < 2) return -1;
  adj_t g;
  if (adj_build(&g, n, m, u, v) != 0) return -2;
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  uint8_t *queued = (uint8_t *)calloc((size_t)m + 1, 1);
  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
  if (!s || !queued || !queue) { free(s); free(queued); free(queue); adj_free(&g); return -2; }
  for (int64_t e = 0; e < m; ++e)
    s[e] = in_out[e] ? common_neighbours(&g, u[e], v[e], in_out) : 0;
  adj_free(&g);
  live_lists_t L;
  if (live_lists_build(&L, n, m, u, v, in_out) != 0) {
    free(s); free(queued); free(queue); return -2;
  }
  int64_t qh = 0, qt = 0;
  for (int64_t e = 0; e < m; ++e)
    if (in_out[e] && s[e] < k - 2) { queued[e] = 1; queue[qt++] = e; }
  while (qh < qt)
    peel_edge_by_search(&L, u, v, queue[qh++], in_out, s, k - 2, queued, queue, &qt);
  free(s); free(queued); free(queue); live_lists_free(&L);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Truss decomposition (Sec. III-B, last paragraph): run the k-truss with      */
/* k = 3 on the whole graph, pass the result on with k + 1, and stop at the    */
/* first empty result.  tau(e) = the largest k whose k-truss contains e        */
/* (every edge is in the 2-truss, which is the whole graph).  *kmax = the      */
/* largest k with a non-empty k-truss: 0 for an empty graph, 2 for a graph     */
/* with edges but no triangle.                                                 */
/*   method 0: bulk rounds (oracle_ktruss_bulk) per level, literally chained.  */
/*   method 1: levelled peeling -- support kept across levels, edges peeled    */
/*             one at a time with incremental decrements (triangle index).     */
/*   method 2: the same levels and peeling rule, with each removed edge's      */
/*             triangles found by searching adjacency lists (no triangle       */
/*             index; the initial support comes from triangle listing).        */
/* ------------------------------------------------------------------------- */
int oracle_truss_decomposition(int32_t n, int64_t m, const int32_t *u,
                               const int32_t *v, int32_t method, int32_t *tau,
                               int32_t *kmax) {
  if (m == 0) { *kmax = 0; return 0; }
  uint8_t *alive = (uint8_t *)malloc((size_t)m + 1);
  if (!alive) return -2;
  memset(alive, 1, (size_t)m);
  for (int64_t e = 0; e < m; ++e) tau[e] = 2;
  int32_t k = 3;
  if (method == 0) {
    for (;; ++k) {
      int32_t r = oracle_ktruss_bulk(n, m, u, v, k, alive);
      if (r < 0) { free(alive); return r; }
      int64_t left = 0;
      for (int64_t e = 0; e < m; ++e)
        if (alive[e]) { tau[e] = k; ++left; }
      if (left == 0) break;
    }
  } else {
    adj_t g;
    tri_index_t t = {0, NULL, NULL};
    live_lists_t L;
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    uint8_t *queued = (uint8_t *)calloc((size_t)m + 1, 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t *live = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!s || !queued || !queue || !live) {
      free(s); free(queued); free(queue); free(live); free(alive);
      return -2;
    }
    if (adj_build(&g, n, m, u, v) != 0) {
      free(s); free(queued); free(queue); free(live); free(alive);
      return -2;
    }
    if (method == 2) {
      int64_t *cnt = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
      int64_t T = cnt ? list_triangles(&g, cnt, NULL, NULL) : -2;
      for (int64_t e = 0; T >= 0 && e < m; ++e) s[e] = (int32_t)cnt[e];
      free(cnt);
      adj_free(&g);
      if (T < 0 || live_lists_build(&L, n, m, u, v, alive) != 0) {
        free(s); free(queued); free(queue); free(live); free(alive);
        return -2;
      }
    } else {
      if (tri_index_build(&g, &t) != 0) {
        tri_index_free(&t); adj_free(&g);
        free(s); free(queued); free(queue); free(live); free(alive);
        return -2;
      }
      adj_free(&g);
      present_support(&t, alive, s);
    }
    int64_t nlive = m;
    for (int64_t e = 0; e < m; ++e) live[e] = e;
    for (;; ++k) {
      int64_t qh = 0, qt = 0;
      for (int64_t i = 0; i < nlive; ++i) {
        int64_t e = live[i];
        if (s[e] < k - 2) { queued[e] = 1; queue[qt++] = e; }
      }
      while (qh < qt) {
        if (method == 2)
          peel_edge_by_search(&L, u, v, queue[qh++], alive, s, k - 2, queued, queue, &qt);
        else
          peel_edge(&t, queue[qh++], alive, s, k - 2, queued, queue, &qt);
      }
      int64_t w = 0;
      for (int64_t i = 0; i < nlive; ++i)
        if (alive[live[i]]) { tau[live[i]] = k; live[w++] = live[i]; }
      nlive = w;
      if (nlive == 0) break;
    }
    free(s); free(queued); free(queue); free(live);
    if (method == 2) live_lists_free(&L);
    else tri_index_free(&t);
  }
  *kmax = k - 1;
  free(alive);
  return 0;
}
