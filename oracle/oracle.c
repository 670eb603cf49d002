/*
 * CPU oracle for exact butterfly counts.  TEST INFRASTRUCTURE ONLY: it is used
 * by the tests, the smoke check and the CPU-baseline leg of the benchmark, and
 * never by the GPU library, which shares no code with it.
 *
 * Plain definitions, written out (Wang, Lin, Qin, Zhang, Zhang, "Efficient
 * Butterfly Counting for Large Bipartite Networks"):
 *
 *   per vertex  (Lemma 1, Eq. 1):  B_x = sum over 2-hop neighbours y of x of
 *                                        C(|N(x) & N(y)|, 2)
 *   total       (Lemma 1, Eq. 2):  B_G = 1/2 sum over one layer of B_x
 *   per edge    (Section 6.1, Eq. 8): B_(u,v) = sum over w in N(v), w != u,
 *                                        of (|N(u) & N(w)| - 1)
 *   processed wedges of BFC-VP (Algorithm 2 with Definition 3): the number of
 *   wedges (u, v, w) with p(v) < p(u) and p(w) < p(u); of BFC-VP++
 *   (Algorithm 3): those with p(w) > p(u) and p(w) > p(v).
 *   caterpillars (Section 1, bipartite clustering coefficient 4 B_G / C_G):
 *   the three-paths (x, y, z, t); each has one middle edge (y, z), whose ends
 *   extend it in (d_y - 1)(d_z - 1) ways, so C_G = sum over edges of that.
 *
 * Intersections are full (no priority filter); each start vertex gets a dense
 * int32 counter over its own layer.  All sums are int64; C(c,2) is c(c-1)/2.
 * OpenMP splits start vertices over threads; every thread keeps its own
 * counters and the results are per-vertex / per-edge values or an int64 sum,
 * so the output does not depend on the thread count.
 *
 * Input: edges int32 [m][2] = (upper id, lower id), ids 0-based per layer.
 * Return codes: 0 ok, -1 bad argument, -2 id out of range, -3 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
  int64_t n;       /* number of source vertices */
  int64_t* off;    /* [n+1] */
  int32_t* nbr;    /* [m] neighbour id in the other layer */
  int32_t* eid;    /* [m] input edge index */
} side_csr;

typedef struct {
  side_csr up;     /* upper vertex -> lower neighbours */
  side_csr lo;     /* lower vertex -> upper neighbours */
  int64_t m;
} bigraph;

static void free_side(side_csr* s) { free(s->off); free(s->nbr); free(s->eid); memset(s, 0, sizeof(*s)); }
static void free_graph(bigraph* g) { free_side(&g->up); free_side(&g->lo); }

/* counting sort of edges by one endpoint; lists keep input order */
static int make_side(side_csr* s, const int32_t* edges, int64_t m, int64_t n, int key_col) {
  s->n = n;
  s->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  s->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  s->eid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  if (!s->off || !s->nbr || !s->eid) return -3;
  for (int64_t i = 0; i < m; ++i) s->off[edges[2 * i + key_col] + 1]++;
  for (int64_t x = 0; x < n; ++x) s->off[x + 1] += s->off[x];
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!cur) return -3;
  memcpy(cur, s->off, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i) {
    int64_t k = cur[edges[2 * i + key_col]]++;
    s->nbr[k] = edges[2 * i + (1 - key_col)];
    s->eid[k] = (int32_t)i;
  }
  free(cur);
  return 0;
}

static int load_graph(bigraph* g, const int32_t* edges, int64_t m, int64_t nU, int64_t nL) {
  memset(g, 0, sizeof(*g));
  if (m < 0 || nU < 0 || nL < 0 || (m > 0 && !edges) || m >= ((int64_t)1 << 31)) return -1;
  for (int64_t i = 0; i < m; ++i) {
    if (edges[2 * i] < 0 || edges[2 * i] >= nU || edges[2 * i + 1] < 0 || edges[2 * i + 1] >= nL) return -2;
  }
  g->m = m;
  int rc = make_side(&g->up, edges, m, nU, 0);
  if (!rc) rc = make_side(&g->lo, edges, m, nL, 1);
  if (rc) free_graph(g);
  return rc;
}

static int64_t sum_deg_sq(const side_csr* s) {
  int64_t t = 0;
  for (int64_t x = 0; x < s->n; ++x) { int64_t d = s->off[x + 1] - s->off[x]; t += d * d; }
  return t;
}

static inline int64_t choose2(int64_t c) { return c * (c - 1) / 2; }

/*
 * Dense counting of |N(s) & N(w)| for one start s: walks s -> v -> w over
 * the start layer S and the middle layer M, skipping w == s.  Distinct ends
 * are listed in `touched`; returns how many.
 */
static int64_t count_common(const side_csr* S, const side_csr* M, int64_t s, int32_t* cnt, int32_t* touched) {
  int64_t nt = 0;
  for (int64_t a = S->off[s]; a < S->off[s + 1]; ++a) {
    int64_t v = S->nbr[a];
    for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b) {
      int32_t w = M->nbr[b];
      if (w == s) continue;
      if (cnt[w]++ == 0) touched[nt++] = w;
    }
  }
  return nt;
}

/* Eq. 1 for every vertex of layer S (middles in layer M). */
static int vertex_counts(const side_csr* S, const side_csr* M, int64_t* out, int nthreads) {
  int failed = 0;
#pragma omp parallel num_threads(nthreads)
  {
    int32_t* cnt = (int32_t*)calloc((size_t)(S->n > 0 ? S->n : 1), sizeof(int32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->n > 0 ? S->n : 1));
    if (!cnt || !touched) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp barrier
    if (!failed) {
#pragma omp for schedule(dynamic, 64)
      for (int64_t s = 0; s < S->n; ++s) {
        int64_t nt = count_common(S, M, s, cnt, touched);
        int64_t acc = 0;
        for (int64_t t = 0; t < nt; ++t) { acc += choose2(cnt[touched[t]]); cnt[touched[t]] = 0; }
        out[s] = acc;
      }
    }
    free(cnt); free(touched);
  }
  return failed ? -3 : 0;
}

/* Eq. 8 for every edge, walked from the start layer S. */
static int edge_counts(const side_csr* S, const side_csr* M, int64_t* out, int nthreads) {
  int failed = 0;
#pragma omp parallel num_threads(nthreads)
  {
    int32_t* cnt = (int32_t*)calloc((size_t)(S->n > 0 ? S->n : 1), sizeof(int32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->n > 0 ? S->n : 1));
    if (!cnt || !touched) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp barrier
    if (!failed) {
#pragma omp for schedule(dynamic, 64)
      for (int64_t s = 0; s < S->n; ++s) {
        int64_t nt = count_common(S, M, s, cnt, touched);
        for (int64_t a = S->off[s]; a < S->off[s + 1]; ++a) {
          int64_t v = S->nbr[a];
          int64_t acc = 0;
          for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b) {
            int32_t w = M->nbr[b];
            if (w != s) acc += (int64_t)cnt[w] - 1;
          }
          out[S->eid[a]] = acc;
        }
        for (int64_t t = 0; t < nt; ++t) cnt[touched[t]] = 0;
      }
    }
    free(cnt); free(touched);
  }
  return failed ? -3 : 0;
}

/* ------------------------------------------------------------- public API */

/* B_x for every upper (side 0) or lower (side 1) vertex, Eq. 1. */
int orc_vertex_counts(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int side, int64_t* out,
                      int nthreads) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  rc = side == 0 ? vertex_counts(&g.up, &g.lo, out, nthreads) : vertex_counts(&g.lo, &g.up, out, nthreads);
  free_graph(&g);
  return rc;
}

/*
 * B_G, Eq. 2: half the sum of B_x over one layer.  The layer is picked by the
 * sum-of-squared-degrees rule of the layer-based baseline (Algorithm 1): start
 * from U unless sum_U d^2 < sum_L d^2.  Either layer gives the same value.
 * side_used reports the layer (0 upper, 1 lower); force_side >= 0 overrides.
 */
int orc_total(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int force_side, int nthreads,
              int64_t* total, int* side_used) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int side = sum_deg_sq(&g.up) < sum_deg_sq(&g.lo) ? 1 : 0;
  if (force_side == 0 || force_side == 1) side = force_side;
  const side_csr* S = side == 0 ? &g.up : &g.lo;
  const side_csr* M = side == 0 ? &g.lo : &g.up;
  int64_t* per = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S->n > 0 ? S->n : 1));
  if (!per) { free_graph(&g); return -3; }
  rc = vertex_counts(S, M, per, nthreads);
  int64_t sum = 0;
  for (int64_t x = 0; x < S->n; ++x) sum += per[x];
  free(per);
  free_graph(&g);
  if (rc) return rc;
  if (sum & 1) return -4; /* impossible for a simple graph: each butterfly holds two vertices of a layer */
  *total = sum / 2;
  if (side_used) *side_used = side;
  return 0;
}

/* B_e for every edge in input order, Eq. 8, from the cheaper start layer
 * (or force_side). */
int orc_edge_counts(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int force_side, int nthreads,
                    int64_t* out) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int side = sum_deg_sq(&g.up) < sum_deg_sq(&g.lo) ? 1 : 0;
  if (force_side == 0 || force_side == 1) side = force_side;
  rc = side == 0 ? edge_counts(&g.up, &g.lo, out, nthreads) : edge_counts(&g.lo, &g.up, out, nthreads);
  free_graph(&g);
  return rc;
}

/* Eq. 1 for the listed vertices xs[0..k) of layer `side` only (a sample of
 * starts, for timing the oracle on part of a large graph). */
int orc_vertex_counts_subset(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int side,
                             const int64_t* xs, int64_t k, int64_t* out, int nthreads) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  const side_csr* S = side == 0 ? &g.up : &g.lo;
  const side_csr* M = side == 0 ? &g.lo : &g.up;
  for (int64_t i = 0; i < k; ++i) if (xs[i] < 0 || xs[i] >= S->n) { free_graph(&g); return -1; }
  int failed = 0;
#pragma omp parallel num_threads(nthreads)
  {
    int32_t* cnt = (int32_t*)calloc((size_t)(S->n > 0 ? S->n : 1), sizeof(int32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->n > 0 ? S->n : 1));
    if (!cnt || !touched) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp barrier
    if (!failed) {
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < k; ++i) {
        int64_t s = xs[i];
        int64_t nt = count_common(S, M, s, cnt, touched);
        int64_t acc = 0;
        for (int64_t t = 0; t < nt; ++t) { acc += choose2(cnt[touched[t]]); cnt[touched[t]] = 0; }
        out[i] = acc;
      }
    }
    free(cnt); free(touched);
  }
  free_graph(&g);
  return failed ? -3 : 0;
}

/* ------------------------------------------------ single-vertex / edge */

/* Handle for repeated single-vertex and single-edge queries on one graph. */
typedef struct { bigraph g; } orc_graph;

orc_graph* orc_open(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int* rc_out) {
  orc_graph* h = (orc_graph*)malloc(sizeof(orc_graph));
  if (!h) { if (rc_out) *rc_out = -3; return NULL; }
  int rc = load_graph(&h->g, edges, m, nU, nL);
  if (rc_out) *rc_out = rc;
  if (rc) { free(h); return NULL; }
  return h;
}

void orc_close(orc_graph* h) { if (h) { free_graph(&h->g); free(h); } }

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Eq. 1 for one vertex x of layer `side`: gather every 2-hop end (with
 * repetition), sort, and add C(run length, 2) per distinct end != x. */
int64_t orc_vertex_one(const orc_graph* h, int side, int64_t x) {
  const side_csr* S = side == 0 ? &h->g.up : &h->g.lo;
  const side_csr* M = side == 0 ? &h->g.lo : &h->g.up;
  if (x < 0 || x >= S->n) return -1;
  int64_t k = 0;
  for (int64_t a = S->off[x]; a < S->off[x + 1]; ++a) { int64_t v = S->nbr[a]; k += M->off[v + 1] - M->off[v]; }
  int32_t* ends = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  if (!ends) return -3;
  int64_t e = 0;
  for (int64_t a = S->off[x]; a < S->off[x + 1]; ++a) {
    int64_t v = S->nbr[a];
    for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b) if (M->nbr[b] != x) ends[e++] = M->nbr[b];
  }
  qsort(ends, (size_t)e, sizeof(int32_t), cmp_i32);
  int64_t acc = 0;
  for (int64_t i = 0; i < e;) {
    int64_t j = i;
    while (j < e && ends[j] == ends[i]) ++j;
    acc += choose2(j - i);
    i = j;
  }
  free(ends);
  return acc;
}

/* Eq. 8 for the edge (u, v): sum over w in N(v), w != u, of |N(u) & N(w)| - 1,
 * each intersection counted by binary search in the sorted copy of N(u). */
int64_t orc_edge_one(const orc_graph* h, int64_t u, int64_t v) {
  const side_csr* U = &h->g.up;
  const side_csr* L = &h->g.lo;
  if (u < 0 || u >= U->n || v < 0 || v >= L->n) return -1;
  int64_t du = U->off[u + 1] - U->off[u];
  int32_t* nu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(du > 0 ? du : 1));
  if (!nu) return -3;
  memcpy(nu, U->nbr + U->off[u], sizeof(int32_t) * (size_t)du);
  qsort(nu, (size_t)du, sizeof(int32_t), cmp_i32);
  int present = bsearch(&(int32_t){(int32_t)v}, nu, (size_t)du, sizeof(int32_t), cmp_i32) != NULL;
  int64_t acc = 0;
  if (present) {
    for (int64_t b = L->off[v]; b < L->off[v + 1]; ++b) {
      int64_t w = L->nbr[b];
      if (w == u) continue;
      int64_t common = 0;
      for (int64_t c = U->off[w]; c < U->off[w + 1]; ++c)
        if (bsearch(&U->nbr[c], nu, (size_t)du, sizeof(int32_t), cmp_i32)) ++common;
      acc += common - 1;
    }
  }
  free(nu);
  return present ? acc : -2;
}

/* ----------------------------------------------- BFC-VP processed wedges */

/* Global id of Section 2: lower v -> v, upper u -> nL + u (so every upper id
 * exceeds every lower id).  Priority (Definition 3): higher degree first, ties
 * broken by the larger id. */
typedef struct { int64_t deg; int64_t id; } prio_key;

static int cmp_prio(const void* a, const void* b) {
  const prio_key* x = (const prio_key*)a;
  const prio_key* y = (const prio_key*)b;
  if (x->deg != y->deg) return (x->deg > y->deg) - (x->deg < y->deg);
  return (x->id > y->id) - (x->id < y->id);
}

/* p[gid] in [0, n): position in ascending priority order. */
static int priorities(const bigraph* g, int64_t* p) {
  int64_t nL = g->lo.n, nU = g->up.n, n = nL + nU;
  prio_key* keys = (prio_key*)malloc(sizeof(prio_key) * (size_t)(n > 0 ? n : 1));
  if (!keys) return -3;
  for (int64_t v = 0; v < nL; ++v) { keys[v].deg = g->lo.off[v + 1] - g->lo.off[v]; keys[v].id = v; }
  for (int64_t u = 0; u < nU; ++u) { keys[nL + u].deg = g->up.off[u + 1] - g->up.off[u]; keys[nL + u].id = nL + u; }
  qsort(keys, (size_t)n, sizeof(prio_key), cmp_prio);
  for (int64_t r = 0; r < n; ++r) p[keys[r].id] = r;
  free(keys);
  return 0;
}

int orc_priorities(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int64_t* p_out) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  rc = priorities(&g, p_out);
  free_graph(&g);
  return rc;
}

/*
 * Wedges processed by BFC-VP (Algorithm 2): for every start u, every
 * neighbour v with p(v) < p(u), every neighbour w of v with p(w) < p(u).
 * per_start (nullable, [nL + nU] by global id) receives each start's count.
 */
int orc_vp_wedges(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int nthreads, int64_t* total,
                  int64_t* per_start) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int64_t n = nU + nL;
  int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!p) { free_graph(&g); return -3; }
  rc = priorities(&g, p);
  int64_t sum = 0;
  if (!rc) {
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : sum) num_threads(nthreads)
    for (int64_t x = 0; x < n; ++x) {
      int upper = x >= nL;
      const side_csr* S = upper ? &g.up : &g.lo;
      const side_csr* M = upper ? &g.lo : &g.up;
      int64_t s = upper ? x - nL : x;
      int64_t mid_off = upper ? 0 : nL;  /* middle layer's global-id offset */
      int64_t end_off = upper ? nL : 0;  /* end layer's global-id offset */
      int64_t w_here = 0;
      for (int64_t a = S->off[s]; a < S->off[s + 1]; ++a) {
        int64_t v = S->nbr[a];
        if (p[mid_off + v] >= p[x]) continue;
        for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b)
          if (p[end_off + M->nbr[b]] < p[x]) ++w_here;
      }
      if (per_start) per_start[x] = w_here;
      sum += w_here;
    }
  }
  free(p);
  free_graph(&g);
  if (!rc) *total = sum;
  return rc;
}

/*
 * Wedges processed by BFC-VP++ (Algorithm 3): for every start u, every
 * neighbour v (no priority test on the middle), every neighbour w of v with
 * p(w) > p(u) and p(w) > p(v): the end outranks both other vertices.
 * Lemma 3 states that this equals the count of Algorithm 2.  per_start
 * (nullable, [nL + nU] by global id) receives each start's count.
 */
int orc_vpp_wedges(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int nthreads, int64_t* total,
                   int64_t* per_start) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int64_t n = nU + nL;
  int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!p) { free_graph(&g); return -3; }
  rc = priorities(&g, p);
  int64_t sum = 0;
  if (!rc) {
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : sum) num_threads(nthreads)
    for (int64_t x = 0; x < n; ++x) {
      int upper = x >= nL;
      const side_csr* S = upper ? &g.up : &g.lo;
      const side_csr* M = upper ? &g.lo : &g.up;
      int64_t s = upper ? x - nL : x;
      int64_t mid_off = upper ? 0 : nL;
      int64_t end_off = upper ? nL : 0;
      int64_t w_here = 0;
      for (int64_t a = S->off[s]; a < S->off[s + 1]; ++a) {
        int64_t v = S->nbr[a];
        int64_t top = p[mid_off + v] > p[x] ? p[mid_off + v] : p[x];
        for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b)
          if (p[end_off + M->nbr[b]] > top) ++w_here;
      }
      if (per_start) per_start[x] = w_here;
      sum += w_here;
    }
  }
  free(p);
  free_graph(&g);
  if (!rc) *total = sum;
  return rc;
}

/*
 * The count_wedge map of Algorithm 2 for one start (global id `start`):
 * ends[i] (global ids, ascending) and counts[i].  Returns the number of
 * distinct ends, or a negative code; at most `cap` entries are written.
 */
int64_t orc_vp_count_wedge(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int64_t start, int64_t* ends,
                           int64_t* counts, int64_t cap) {
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int64_t n = nU + nL;
  if (start < 0 || start >= n) { free_graph(&g); return -1; }
  int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* c = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  if (!p || !c) { free(p); free(c); free_graph(&g); return -3; }
  priorities(&g, p);
  int upper = start >= nL;
  const side_csr* S = upper ? &g.up : &g.lo;
  const side_csr* M = upper ? &g.lo : &g.up;
  int64_t s = upper ? start - nL : start;
  int64_t mid_off = upper ? 0 : nL, end_off = upper ? nL : 0;
  for (int64_t a = S->off[s]; a < S->off[s + 1]; ++a) {
    int64_t v = S->nbr[a];
    if (p[mid_off + v] >= p[start]) continue;
    for (int64_t b = M->off[v]; b < M->off[v + 1]; ++b) {
      int64_t w = end_off + M->nbr[b];
      if (p[w] < p[start]) c[w]++;
    }
  }
  int64_t k = 0;
  for (int64_t w = 0; w < n; ++w) {
    if (c[w]) { if (k < cap) { ends[k] = w; counts[k] = c[w]; } ++k; }
  }
  free(p); free(c);
  free_graph(&g);
  return k;
}

/* C_G = sum over edges (u, v) of (d_u - 1)(d_v - 1) (caterpillars). */
int orc_caterpillars(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int64_t* out) {
  if (!out) return -1;
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int64_t c = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int64_t du = g.up.off[edges[2 * i] + 1] - g.up.off[edges[2 * i]];
    const int64_t dv = g.lo.off[edges[2 * i + 1] + 1] - g.lo.off[edges[2 * i + 1]];
    c += (du - 1) * (dv - 1);
  }
  free_graph(&g);
  *out = c;
  return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------- k-wing */

/* The k-wing (Section 1, computing k-wing in bipartite graphs): the largest
 * subgraph in which every edge lies in at least k butterflies.  Following the
 * peeling the paper describes: count the butterflies of every edge (Eq. 8),
 * then repeatedly remove the remaining edge with the fewest butterflies while
 * that number is below k.  Removing e = (u, v) destroys exactly the
 * butterflies (u, v, u2, v2) with u2 in N(v), v2 in N(u) and (u2, v2) a
 * remaining edge; each of its three other edges loses one.  Edges below k wait
 * in a binary min-heap on (count, edge index) with a position index, so a
 * count that drops moves its edge up in place.
 *
 * Output: in_wing[i] = 1 for the input edges of the k-wing, else 0; counts[i]
 * (may be NULL) the butterflies of edge i within the k-wing, 0 outside it.
 * *removed_out (may be NULL) receives the number of removed edges. */
typedef struct {
  int32_t* heap;   /* edge indices */
  int32_t* pos;    /* heap position of each edge, -1 when absent */
  int64_t n;
  const int64_t* key;
} wing_heap;

static int heap_less(const wing_heap* h, int32_t a, int32_t b) {
  return h->key[a] < h->key[b] || (h->key[a] == h->key[b] && a < b);
}

static void heap_up(wing_heap* h, int64_t i) {
  int32_t e = h->heap[i];
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!heap_less(h, e, h->heap[p])) break;
    h->heap[i] = h->heap[p];
    h->pos[h->heap[i]] = (int32_t)i;
    i = p;
  }
  h->heap[i] = e;
  h->pos[e] = (int32_t)i;
}

static void heap_down(wing_heap* h, int64_t i) {
  int32_t e = h->heap[i];
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->n) break;
    if (c + 1 < h->n && heap_less(h, h->heap[c + 1], h->heap[c])) ++c;
    if (!heap_less(h, h->heap[c], e)) break;
    h->heap[i] = h->heap[c];
    h->pos[h->heap[i]] = (int32_t)i;
    i = c;
  }
  h->heap[i] = e;
  h->pos[e] = (int32_t)i;
}

static void heap_push_or_raise(wing_heap* h, int32_t e) {
  if (h->pos[e] >= 0) { heap_up(h, h->pos[e]); return; }
  h->heap[h->n] = e;
  heap_up(h, h->n++);
}

static int32_t heap_pop(wing_heap* h) {
  int32_t top = h->heap[0];
  h->pos[top] = -1;
  if (--h->n > 0) {
    h->heap[0] = h->heap[h->n];
    heap_down(h, 0);
  }
  return top;
}

typedef struct { int32_t nbr; int32_t eid; } nbr_eid;

static int cmp_nbr_eid(const void* a, const void* b) {
  int32_t x = ((const nbr_eid*)a)->nbr, y = ((const nbr_eid*)b)->nbr;
  return (x > y) - (x < y);
}

int orc_k_wing(const int32_t* edges, int64_t m, int64_t nU, int64_t nL, int64_t k, int nthreads,
               uint8_t* in_wing, int64_t* counts, int64_t* removed_out) {
  if (!in_wing && m > 0) return -1;
  bigraph g;
  int rc = load_graph(&g, edges, m, nU, nL);
  if (rc) return rc;
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  uint8_t* alive = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
  wing_heap h = {(int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)),
                 (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)), 0, NULL};
  /* both layers' lists sorted by neighbour, with edge indices */
  nbr_eid* su = (nbr_eid*)malloc(sizeof(nbr_eid) * (size_t)(m > 0 ? m : 1));
  nbr_eid* sl = (nbr_eid*)malloc(sizeof(nbr_eid) * (size_t)(m > 0 ? m : 1));
  if (!cnt || !alive || !h.heap || !h.pos || !su || !sl) { rc = -3; goto done; }
  rc = edge_counts(&g.up, &g.lo, cnt, nthreads > 0 ? nthreads : 1);
  if (rc) goto done;
  for (int64_t a = 0; a < m; ++a) {
    su[a].nbr = g.up.nbr[a]; su[a].eid = g.up.eid[a];
    sl[a].nbr = g.lo.nbr[a]; sl[a].eid = g.lo.eid[a];
  }
  for (int64_t x = 0; x < nU; ++x)
    qsort(su + g.up.off[x], (size_t)(g.up.off[x + 1] - g.up.off[x]), sizeof(nbr_eid), cmp_nbr_eid);
  for (int64_t x = 0; x < nL; ++x)
    qsort(sl + g.lo.off[x], (size_t)(g.lo.off[x + 1] - g.lo.off[x]), sizeof(nbr_eid), cmp_nbr_eid);
  h.key = cnt;
  for (int64_t i = 0; i < m; ++i) {
    alive[i] = 1;
    h.pos[i] = -1;
    if (cnt[i] < k) heap_push_or_raise(&h, (int32_t)i);
  }
  int64_t removed = 0;
  while (h.n > 0) {
    const int32_t e = heap_pop(&h);  /* the remaining edge with the fewest butterflies, below k */
    const int32_t u = edges[2 * e], v = edges[2 * e + 1];
    alive[e] = 0;
    ++removed;
    /* every butterfly (u, v, u2, v2) still present loses e */
    for (int64_t b = g.lo.off[v]; b < g.lo.off[v + 1]; ++b) {
      const int32_t u2 = sl[b].nbr, e1 = sl[b].eid;   /* e1 = (u2, v) */
      if (u2 == u || !alive[e1]) continue;
      for (int64_t c = g.up.off[u]; c < g.up.off[u + 1]; ++c) {
        const int32_t v2 = su[c].nbr, e2 = su[c].eid;  /* e2 = (u, v2) */
        if (v2 == v || !alive[e2]) continue;
        int64_t lo = g.up.off[u2], hi = g.up.off[u2 + 1];
        while (lo < hi) {
          int64_t mid = lo + (hi - lo) / 2;
          if (su[mid].nbr < v2) lo = mid + 1; else hi = mid;
        }
        if (lo == g.up.off[u2 + 1] || su[lo].nbr != v2) continue;
        const int32_t e3 = su[lo].eid;                 /* e3 = (u2, v2) */
        if (!alive[e3]) continue;
        const int32_t hit[3] = {e1, e2, e3};
        for (int t = 0; t < 3; ++t) {
          if (--cnt[hit[t]] < k) heap_push_or_raise(&h, hit[t]);
        }
      }
    }
  }
  for (int64_t i = 0; i < m; ++i) {
    in_wing[i] = alive[i];
    if (counts) counts[i] = alive[i] ? cnt[i] : 0;
  }
  if (removed_out) *removed_out = removed;
done:
  free(cnt); free(alive); free(h.heap); free(h.pos); free(su); free(sl);
  free_graph(&g);
  return rc;
}
