/*
 * fl_oracle.c -- plain, slow, single-threaded CPU oracle for sketch-based
 * facility location on graphs (Scalable Facility Location for Massive Graphs
 * on Pregel-like Systems, arXiv 1503.03635).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library; every step below is written out from the
 * paper (and, where the paper is silent, from the stated reading).
 *
 * Arithmetic: IEEE-754 double, round-to-nearest, compiled with
 * -ffp-contract=off and without fast-math, so every line is one rounding per
 * operation in the order written.  Distances are exact integers (uint64 inside,
 * reported as uint32).
 *
 * Contents (each function cites the passage it follows):
 *   ranks ........ seeded bijection r(v) ("r(u) is the hash of u", Sec. 3.3,
 *                  Alg. 1) and MIS priorities pi(f) (Sec. 4.3)
 *   ADS .......... (i) brute force = Alg. 1 with the (distance, id) order,
 *                  (ii) pruned Dijkstra, (iii) Alg. 2 synchronous rounds with
 *                  the CleanUp applied every superstep
 *   HIP weights .. historic-inverse-probability adjusted weights (Sec. 3.3,
 *                  cited there to Cohen's ADS paper)
 *   solve ........ gamma and alpha_0 (Sec. 4.1), radius ladder R (Sec. 4.2),
 *                  OpenFacilities with Eq. 2 / Eq. 3 (Alg. 5), freezing with
 *                  Alg. 3's (1+eps)alpha(c) rule, end phase (Alg. 3/Alg. 4),
 *                  MIS on H-bar per rung (Sec. 4.3, Alg. 6), assignment and
 *                  objective (Sec. 3.1)
 *   exhaustive ... OPT over all non-empty facility subsets (tiny n only)
 *
 * Directed graphs (Sec. 3.1 considers them; the algorithm is adapted to them
 * without the guarantee, Sec. 4.4): d(u, v) is the shortest path along arcs
 * from u to v.  Entries travel along arcs (Alg. 2 sends (u, d + e(u,v)) to
 * the out-neighbours), so the sketch of v holds vertices u that reach v, at
 * d(u, v); a facility's estimate counts the clients that can reach it; a
 * client is served by, frozen by and in conflict through facilities it can
 * reach, at d(c, f).  Searches for distances into a vertex run on the
 * reversed arcs.  On an undirected graph both directions coincide.
 *
 * Readings of passages that are silent or ambiguous are listed in the design
 * notes; the short form of each is repeated at the point of use.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ERANGE 2
#define ORC_ENOMEM 3
#define ORC_EINTERNAL 99

#define ORC_INF64 UINT64_MAX
#define ORC_NONE 0xFFFFFFFFu
#define RUNG_NONE 0xFFFFFFFFu
#define RUNG_GUARD 0xFFFFFFFEu
#define RUNG_END 0xFFFFFFFDu
#define NOT_FACILITY 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Input graph (host pointers).                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n;
  uint64_t n_arcs;
  const uint64_t *row_ptr; /* [n+1] */
  const uint32_t *col;     /* [n_arcs] */
  const uint32_t *w;       /* [n_arcs] or NULL = unit weights */
  const uint32_t *fac_cost;/* [n], NOT_FACILITY marks non-facilities; may be NULL for ADS-only calls */
  const uint8_t *is_client;/* [n] or NULL = every vertex is a client */
  uint32_t directed;       /* 0: symmetric CSR of an undirected graph;
                              1: rows are the out-arcs of a directed graph */
} orc_graph;

typedef struct {
  uint64_t *off;  /* [n+1] */
  uint32_t *rank; /* [total] */
  uint32_t *dist; /* [total] */
  uint32_t *id;   /* [total] vertex id of each entry */
} orc_sketch;

static inline uint32_t arcw(const orc_graph *g, uint64_t i) { return g->w ? g->w[i] : 1u; }

/* The graph with every arc turned around: row v lists the u with an arc
 * u -> v (increasing u), with that arc's weight.  A search from s over it
 * yields d(u, s), the distance INTO s.  An undirected graph is its own
 * reverse; then nothing is allocated. */
typedef struct { orc_graph g; uint64_t *rp; uint32_t *col, *w; } orc_rev;

static int reverse_graph(const orc_graph *g, orc_rev *r) {
  r->g = *g;
  r->rp = NULL; r->col = NULL; r->w = NULL;
  if (!g->directed) return 0;
  uint32_t n = g->n;
  uint64_t m = g->n_arcs;
  r->rp = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
  r->col = (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t));
  r->w = g->w ? (uint32_t *)malloc((size_t)(m ? m : 1) * sizeof(uint32_t)) : NULL;
  uint64_t *fill = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
  if (!r->rp || !r->col || (g->w && !r->w) || !fill) return 1;
  for (uint64_t i = 0; i < m; i++) r->rp[g->col[i] + 1]++;
  for (uint32_t v = 0; v < n; v++) r->rp[v + 1] += r->rp[v];
  for (uint32_t v = 0; v < n; v++) fill[v] = r->rp[v];
  for (uint32_t u = 0; u < n; u++)
    for (uint64_t i = g->row_ptr[u]; i < g->row_ptr[u + 1]; i++) {
      uint64_t p = fill[g->col[i]]++;
      r->col[p] = u;
      if (r->w) r->w[p] = g->w[i];
    }
  free(fill);
  r->g.row_ptr = r->rp;
  r->g.col = r->col;
  r->g.w = r->w;
  return 0;
}
static void reverse_free(orc_rev *r) { free(r->rp); free(r->col); free(r->w); }

/* ------------------------------------------------------------------------ */
/* Ranks: a seeded bijection on 32-bit integers.                             */
/* The paper only says the rank of u is "the hash of u" (Alg. 1) and that MIS */
/* priorities are drawn from [1, n^3] and unique with high probability         */
/* (Sec. 4.3).  Reading: both are bijections of the vertex id, so ranks and    */
/* priorities are distinct for certain and a rank can be mapped back to its    */
/* vertex.  Construction: two rounds of the public-domain MurmurHash3 32-bit   */
/* finaliser ("fmix32"), each preceded by an xor with a 32-bit key; the keys   */
/* come from Vigna's public-domain SplitMix64 mixer applied to seed^1 (ranks)  */
/* and seed^2 (priorities).  Every step (xor with a key, xorshift, odd         */
/* multiply) is invertible, which gives the inverse below.                     */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* inverse of y = x ^ (x >> s): x = y ^ (y >> s) ^ (y >> 2s) ^ ... */
static uint32_t unshift(uint32_t y, int s) {
  uint32_t x = y;
  for (int t = s; t < 32; t += s) x ^= y >> t;
  return x;
}

/* inverse of an odd number modulo 2^32 by Newton iteration */
static uint32_t inv_odd(uint32_t c) {
  uint32_t x = c;
  for (int i = 0; i < 5; i++) x *= 2u - c * x;
  return x;
}

static uint32_t unfmix32(uint32_t h) {
  h = unshift(h, 16);
  h *= inv_odd(0xc2b2ae35u);
  h = unshift(h, 13);
  h *= inv_odd(0x85ebca6bu);
  h = unshift(h, 16);
  return h;
}

uint32_t orc_perm(uint32_t v, uint64_t key) {
  uint32_t k1 = (uint32_t)key, k2 = (uint32_t)(key >> 32);
  uint32_t x = fmix32(v ^ k1);
  return fmix32(x ^ k2);
}

uint32_t orc_perm_inv(uint32_t r, uint64_t key) {
  uint32_t k1 = (uint32_t)key, k2 = (uint32_t)(key >> 32);
  uint32_t x = unfmix32(r) ^ k2;
  return unfmix32(x) ^ k1;
}

uint64_t orc_rank_key(uint64_t seed) { return orc_splitmix64(seed ^ 1ull); }
uint64_t orc_prio_key(uint64_t seed) { return orc_splitmix64(seed ^ 2ull); }

void orc_ranks(uint32_t n, uint64_t seed, uint32_t *rank, uint32_t *prio) {
  uint64_t kr = orc_rank_key(seed), kp = orc_prio_key(seed);
  for (uint32_t v = 0; v < n; v++) {
    if (rank) rank[v] = orc_perm(v, kr);
    if (prio) prio[v] = orc_perm(v, kp);
  }
}

/* Check that orc_perm_inv inverts orc_perm on the ids [lo, lo + count). */
int orc_perm_check_range(uint64_t key, uint32_t lo, uint64_t count) {
  for (uint64_t i = 0; i < count; i++) {
    uint32_t x = (uint32_t)(lo + i);
    if (orc_perm_inv(orc_perm(x, key), key) != x) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Validation (problem statement, Sec. 3.1: undirected graph, positive       */
/* weights).  Reading: a simple undirected graph given as a symmetric CSR     */
/* with strictly increasing neighbour ids per row, integer weights >= 1, no   */
/* self loops.  A bound keeps every distance and every cost+distance below    */
/* 2^32 - 1: (n-1)*max_w + max_cost < 2^32 - 1, else ERANGE.  A directed      */
/* graph (Sec. 3.1) gives its out-arcs per row, with the same rules except    */
/* symmetry.                                                                   */
/* ------------------------------------------------------------------------ */
static int find_arc(const orc_graph *g, uint32_t u, uint32_t v, uint64_t *pos) {
  uint64_t lo = g->row_ptr[u], hi = g->row_ptr[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  if (lo < g->row_ptr[u + 1] && g->col[lo] == v) { *pos = lo; return 1; }
  return 0;
}

int orc_validate(const orc_graph *g, uint32_t k, double eps) {
  if (!g || g->n == 0 || g->n >= 0xFFFFFFFFu) return ORC_EINVAL;
  if (k == 0) return ORC_EINVAL;
  if (!(eps > 0.0) || !isfinite(eps)) return ORC_EINVAL;
  if (!g->row_ptr || (g->n_arcs && !g->col)) return ORC_EINVAL;
  uint32_t n = g->n;
  if (g->row_ptr[0] != 0 || g->row_ptr[n] != g->n_arcs) return ORC_EINVAL;
  uint64_t maxw = 1;
  for (uint32_t u = 0; u < n; u++) {
    if (g->row_ptr[u + 1] < g->row_ptr[u]) return ORC_EINVAL;
    for (uint64_t i = g->row_ptr[u]; i < g->row_ptr[u + 1]; i++) {
      uint32_t v = g->col[i];
      if (v >= n || v == u) return ORC_EINVAL;
      if (i > g->row_ptr[u] && g->col[i - 1] >= v) return ORC_EINVAL;
      uint32_t wi = arcw(g, i);
      if (wi == 0) return ORC_EINVAL;
      if (wi > maxw) maxw = wi;
    }
  }
  /* symmetry (same arc both ways, same weight) only for undirected input */
  for (uint32_t u = 0; u < n && !g->directed; u++) {
    for (uint64_t i = g->row_ptr[u]; i < g->row_ptr[u + 1]; i++) {
      uint64_t back;
      if (!find_arc(g, g->col[i], u, &back)) return ORC_EINVAL;
      if (arcw(g, back) != arcw(g, i)) return ORC_EINVAL;
    }
  }
  uint64_t maxc = 0;
  if (g->fac_cost)
    for (uint32_t v = 0; v < n; v++)
      if (g->fac_cost[v] != NOT_FACILITY && g->fac_cost[v] > maxc) maxc = g->fac_cost[v];
  unsigned __int128 bound = (unsigned __int128)(n - 1) * maxw + maxc;
  if (bound >= 0xFFFFFFFFull) return ORC_ERANGE;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Binary heap keyed by (key, tie, vertex), lexicographic.                    */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; uint32_t tie, v; } hitem;
typedef struct { hitem *a; size_t n, cap; } heap;

static int hless(hitem x, hitem y) {
  if (x.key != y.key) return x.key < y.key;
  if (x.tie != y.tie) return x.tie < y.tie;
  return x.v < y.v;
}
static int hpush(heap *h, uint64_t key, uint32_t tie, uint32_t v) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? 2 * h->cap : 64;
    hitem *na = (hitem *)realloc(h->a, nc * sizeof(hitem));
    if (!na) return 0;
    h->a = na; h->cap = nc;
  }
  size_t i = h->n++;
  hitem it = {key, tie, v};
  while (i > 0) {
    size_t p = (i - 1) / 2;
    if (!hless(it, h->a[p])) break;
    h->a[i] = h->a[p]; i = p;
  }
  h->a[i] = it;
  return 1;
}
static hitem hpop(heap *h) {
  hitem top = h->a[0], last = h->a[--h->n];
  size_t i = 0;
  for (;;) {
    size_t l = 2 * i + 1, r = l + 1, m = i;
    hitem best = last;
    if (l < h->n && hless(h->a[l], best)) { best = h->a[l]; m = l; }
    if (r < h->n && hless(h->a[r], best)) { best = h->a[r]; m = r; }
    if (m == i) break;
    h->a[i] = h->a[m]; i = m;
  }
  if (h->n) h->a[i] = last;
  return top;
}

/* Single-source Dijkstra; fills dist (ORC_INF64 = unreachable) and, if order
 * is non-NULL, the settled vertices in increasing (distance, id) order.
 * Pops come out in (distance, id) order because every weight is >= 1: all
 * vertices at distance d are pushed with their final label before the first
 * of them is popped. */
static int dijkstra(const orc_graph *g, uint32_t s, uint64_t *dist, uint32_t *order, uint32_t *n_order) {
  heap h = {0};
  for (uint32_t v = 0; v < g->n; v++) dist[v] = ORC_INF64;
  dist[s] = 0;
  if (!hpush(&h, 0, s, s)) return ORC_ENOMEM;
  uint32_t cnt = 0;
  while (h.n) {
    hitem it = hpop(&h);
    if (it.key != dist[it.v]) continue;
    if (order) order[cnt] = it.v;
    cnt++;
    for (uint64_t i = g->row_ptr[it.v]; i < g->row_ptr[it.v + 1]; i++) {
      uint32_t y = g->col[i];
      uint64_t nd = it.key + arcw(g, i);
      if (nd < dist[y]) { dist[y] = nd; if (!hpush(&h, nd, y, y)) { free(h.a); return ORC_ENOMEM; } }
    }
  }
  if (n_order) *n_order = cnt;
  free(h.a);
  return ORC_OK;
}

/* Exported for tests: distances from one source (UINT64_MAX = unreachable). */
int orc_sssp(const orc_graph *g, uint32_t s, uint64_t *dist) { return dijkstra(g, s, dist, NULL, NULL); }

/* Multi-source Dijkstra with lexicographic labels (value, tie).  Each source
 * s carries an initial label (init_val[s], init_tie[s]); a label moves along an
 * arc of the given graph by adding the arc weight to its value.  Result: for
 * every v the minimum over sources of (init_val[s] + d'(s,v), init_tie[s]),
 * d' measured along the given rows; on the reversed graph d'(s,v) = d(v,s).
 * Sources are the v with init_val[v] != ORC_INF64. */
static int msdijkstra(const orc_graph *g, const uint64_t *init_val, const uint32_t *init_tie,
                      uint64_t *val, uint32_t *tie) {
  heap h = {0};
  for (uint32_t v = 0; v < g->n; v++) {
    val[v] = init_val[v];
    tie[v] = init_val[v] == ORC_INF64 ? ORC_NONE : init_tie[v];
    if (init_val[v] != ORC_INF64 && !hpush(&h, val[v], tie[v], v)) { free(h.a); return ORC_ENOMEM; }
  }
  while (h.n) {
    hitem it = hpop(&h);
    if (it.key != val[it.v] || it.tie != tie[it.v]) continue;
    for (uint64_t i = g->row_ptr[it.v]; i < g->row_ptr[it.v + 1]; i++) {
      uint32_t y = g->col[i];
      uint64_t nv = it.key + arcw(g, i);
      if (nv < val[y] || (nv == val[y] && it.tie < tie[y])) {
        val[y] = nv; tie[y] = it.tie;
        if (!hpush(&h, nv, it.tie, y)) { free(h.a); return ORC_ENOMEM; }
      }
    }
  }
  free(h.a);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* ADS definition (Sec. 3.3): the sketch of v keeps (u, d(v,u)) when the rank */
/* of u is below the k-th smallest rank among the vertices listed before u in */
/* increasing distance from v.  Reading of the order: ties in distance are    */
/* broken by vertex id, which does not depend on the seed.  Entries are kept  */
/* sorted by (distance, id).                                                   */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t d; uint32_t id; uint32_t rank; } ent;
typedef struct { ent *a; uint32_t n, cap; } entvec;

static int ev_push(entvec *e, ent x) {
  if (e->n == e->cap) {
    uint32_t nc = e->cap ? 2 * e->cap : 8;
    ent *na = (ent *)realloc(e->a, (size_t)nc * sizeof(ent));
    if (!na) return 0;
    e->a = na; e->cap = nc;
  }
  e->a[e->n++] = x;
  return 1;
}

static int sketch_from_vecs(uint32_t n, entvec *vecs, orc_sketch *out) {
  uint64_t total = 0;
  for (uint32_t v = 0; v < n; v++) total += vecs[v].n;
  out->off = (uint64_t *)malloc((size_t)(n + 1) * sizeof(uint64_t));
  out->rank = (uint32_t *)malloc((size_t)(total ? total : 1) * sizeof(uint32_t));
  out->dist = (uint32_t *)malloc((size_t)(total ? total : 1) * sizeof(uint32_t));
  out->id = (uint32_t *)malloc((size_t)(total ? total : 1) * sizeof(uint32_t));
  if (!out->off || !out->rank || !out->dist || !out->id) return ORC_ENOMEM;
  uint64_t p = 0;
  for (uint32_t v = 0; v < n; v++) {
    out->off[v] = p;
    for (uint32_t j = 0; j < vecs[v].n; j++) {
      if (vecs[v].a[j].d >= 0xFFFFFFFFull) return ORC_ERANGE;
      out->rank[p] = vecs[v].a[j].rank;
      out->dist[p] = (uint32_t)vecs[v].a[j].d;
      out->id[p] = vecs[v].a[j].id;
      p++;
    }
  }
  out->off[n] = p;
  return ORC_OK;
}

void orc_sketch_free(orc_sketch *s) {
  if (!s) return;
  free(s->off); free(s->rank); free(s->dist); free(s->id);
  s->off = NULL; s->rank = s->dist = s->id = NULL;
}

/* Running bottom-k of ranks: sorted ascending array of at most k values. */
typedef struct { uint32_t *v; uint32_t n, k; } bottomk;

/* number of stored ranks smaller than r */
static uint32_t bk_count_below(const bottomk *b, uint32_t r) {
  uint32_t c = 0;
  while (c < b->n && b->v[c] < r) c++;
  return c;
}
/* insert r, keeping the k smallest */
static void bk_insert(bottomk *b, uint32_t r) {
  uint32_t pos = bk_count_below(b, r);
  if (pos >= b->k) return;
  uint32_t last = b->n < b->k ? b->n : b->k - 1;
  for (uint32_t i = last; i > pos; i--) b->v[i] = b->v[i - 1];
  b->v[pos] = r;
  if (b->n < b->k) b->n++;
}

/* (i) Brute force: Alg. 1 run per vertex over the (distance, id) order.  A
 * listed vertex enters the sketch when fewer than k vertices listed before it
 * have a smaller rank; every listed vertex then enters the bottom-k set. */
int orc_ads_brute(const orc_graph *g, const uint32_t *rank, uint32_t k, orc_sketch *out) {
  uint32_t n = g->n;
  orc_rev rv;
  if (reverse_graph(g, &rv)) return ORC_ENOMEM;
  uint64_t *dist = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *order = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint32_t *bkv = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  entvec *vecs = (entvec *)calloc(n, sizeof(entvec));
  if (!dist || !order || !bkv || !vecs) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (uint32_t v = 0; v < n && rc == ORC_OK; v++) {
    uint32_t cnt;
    rc = dijkstra(&rv.g, v, dist, order, &cnt); /* d(u, v) for every u */
    bottomk b = {bkv, 0, k};
    for (uint32_t i = 0; i < cnt && rc == ORC_OK; i++) {
      uint32_t u = order[i];
      if (bk_count_below(&b, rank[u]) < k) {
        ent e = {dist[u], u, rank[u]};
        if (!ev_push(&vecs[v], e)) rc = ORC_ENOMEM;
      }
      bk_insert(&b, rank[u]);
    }
  }
  if (rc == ORC_OK) rc = sketch_from_vecs(n, vecs, out);
  for (uint32_t v = 0; v < n; v++) free(vecs[v].a);
  free(vecs); free(dist); free(order); free(bkv);
  reverse_free(&rv);
  return rc;
}

/* The sketch of one vertex v by the definition (Alg. 1 with the (distance,
 * id) order): Dijkstra from v, vertices in that order, each inserted iff fewer
 * than k earlier ones have a smaller rank.  Entries (rank, distance) in
 * sketch order into out_rank/out_dist (capacity cap); *count receives the
 * size (ORC_ENOMEM if it exceeds cap).  Used to check single sketches of
 * graphs too large for the all-vertex builders. */
int orc_ads_one(const orc_graph *g, const uint32_t *rank, uint32_t k, uint32_t v, uint32_t *out_rank,
                uint32_t *out_dist, uint32_t cap, uint32_t *count) {
  uint32_t n = g->n;
  uint64_t *dist = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *order = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint32_t *bkv = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  orc_rev rv;
  if (!dist || !order || !bkv || reverse_graph(g, &rv)) return ORC_ENOMEM;
  uint32_t cnt;
  int rc = dijkstra(&rv.g, v, dist, order, &cnt); /* d(u, v) for every u */
  bottomk b = {bkv, 0, k};
  uint32_t m = 0;
  for (uint32_t i = 0; i < cnt && rc == ORC_OK; i++) {
    uint32_t u = order[i];
    if (bk_count_below(&b, rank[u]) < k) {
      if (m == cap) rc = ORC_ENOMEM;
      else {
        out_rank[m] = rank[u];
        out_dist[m] = (uint32_t)dist[u];
        m++;
      }
    }
    bk_insert(&b, rank[u]);
  }
  *count = m;
  free(dist); free(order); free(bkv);
  reverse_free(&rv);
  return rc;
}

/* (ii) Pruned Dijkstra: sources in increasing rank; a search from u along
 * the arcs (so d = d(u, x)) that settles x at distance d is pruned at x when the sketch of x already holds k
 * entries that come before (d, id(u)) -- all of them have a smaller rank,
 * since sources are taken by increasing rank.  Otherwise (r(u), d) is inserted
 * at its sorted place and the search continues past x.  relax_count (may be
 * NULL) receives the number of arc relaxations performed; max_sources limits
 * the run to the first sources in rank order (0 = all), for timing only. */
static int ent_before(uint64_t d1, uint32_t id1, uint64_t d2, uint32_t id2) {
  return d1 < d2 || (d1 == d2 && id1 < id2);
}

int orc_ads_pruned_ex(const orc_graph *g, const uint32_t *rank, uint32_t k, orc_sketch *out,
                      uint64_t max_sources, uint64_t *relax_count) {
  uint32_t n = g->n;
  uint32_t *srcs = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint64_t *dist = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *touched = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  entvec *vecs = (entvec *)calloc(n, sizeof(entvec));
  if (!srcs || !dist || !touched || !vecs) return ORC_ENOMEM;
  /* sources sorted by rank: counting via the inverse is not available here, so
   * sort (rank, id) pairs */
  uint64_t *keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  if (!keys) return ORC_ENOMEM;
  for (uint32_t v = 0; v < n; v++) keys[v] = ((uint64_t)rank[v] << 32) | v;
  /* simple heap sort to avoid qsort comparator subtleties */
  {
    heap h = {0};
    for (uint32_t v = 0; v < n; v++)
      if (!hpush(&h, keys[v], 0, v)) return ORC_ENOMEM;
    for (uint32_t i = 0; i < n; i++) srcs[i] = (uint32_t)(hpop(&h).key & 0xFFFFFFFFu);
    free(h.a);
  }
  free(keys);
  for (uint32_t v = 0; v < n; v++) dist[v] = ORC_INF64;
  uint64_t relax = 0;
  uint64_t nsrc = max_sources && max_sources < n ? max_sources : n;
  int rc = ORC_OK;
  heap h = {0};
  for (uint64_t si = 0; si < nsrc && rc == ORC_OK; si++) {
    uint32_t u = srcs[si];
    uint32_t ntouch = 0;
    dist[u] = 0;
    touched[ntouch++] = u;
    h.n = 0;
    if (!hpush(&h, 0, u, u)) { rc = ORC_ENOMEM; break; }
    while (h.n && rc == ORC_OK) {
      hitem it = hpop(&h);
      uint32_t x = it.v;
      if (it.key != dist[x]) continue;
      entvec *sx = &vecs[x];
      /* position of (d, id(u)) among the entries of x */
      uint32_t lo = 0, hi = sx->n;
      while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (ent_before(sx->a[mid].d, sx->a[mid].id, it.key, u)) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= k) continue; /* pruned: k entries of smaller rank come first */
      ent e = {it.key, u, rank[u]};
      if (!ev_push(sx, e)) { rc = ORC_ENOMEM; break; }
      for (uint32_t i = sx->n - 1; i > lo; i--) sx->a[i] = sx->a[i - 1];
      sx->a[lo] = e;
      for (uint64_t i = g->row_ptr[x]; i < g->row_ptr[x + 1]; i++) {
        uint32_t y = g->col[i];
        uint64_t nd = it.key + arcw(g, i);
        relax++;
        if (nd < dist[y]) {
          if (dist[y] == ORC_INF64) touched[ntouch++] = y;
          dist[y] = nd;
          if (!hpush(&h, nd, y, y)) { rc = ORC_ENOMEM; break; }
        }
      }
    }
    for (uint32_t i = 0; i < ntouch; i++) dist[touched[i]] = ORC_INF64;
  }
  free(h.a);
  if (relax_count) *relax_count = relax;
  if (rc == ORC_OK && out) rc = sketch_from_vecs(n, vecs, out);
  for (uint32_t v = 0; v < n; v++) free(vecs[v].a);
  free(vecs); free(srcs); free(dist); free(touched);
  return rc;
}

int orc_ads_pruned(const orc_graph *g, const uint32_t *rank, uint32_t k, orc_sketch *out) {
  return orc_ads_pruned_ex(g, rank, k, out, 0, NULL);
}

/* prune(X) on an explicit multiset of (distance, id, rank) triples:
 * keep, per id, the smallest distance; order by (distance, id); drop an entry
 * when k entries before it have a smaller rank.  Used by Alg. 2 below and
 * exported for the associativity pin. */
static int ent_cmp_id_d(const void *pa, const void *pb) {
  const ent *a = (const ent *)pa, *b = (const ent *)pb;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  if (a->d != b->d) return a->d < b->d ? -1 : 1;
  return 0;
}
static int ent_cmp_d_id(const void *pa, const void *pb) {
  const ent *a = (const ent *)pa, *b = (const ent *)pb;
  if (a->d != b->d) return a->d < b->d ? -1 : 1;
  if (a->id != b->id) return a->id < b->id ? -1 : 1;
  return 0;
}

static uint32_t prune_inplace(ent *x, uint32_t m, uint32_t k, uint32_t *bkbuf) {
  if (m == 0) return 0;
  qsort(x, m, sizeof(ent), ent_cmp_id_d);
  uint32_t u = 0;
  for (uint32_t i = 0; i < m; i++)
    if (u == 0 || x[u - 1].id != x[i].id) x[u++] = x[i];
  qsort(x, u, sizeof(ent), ent_cmp_d_id);
  bottomk b = {bkbuf, 0, k};
  uint32_t o = 0;
  for (uint32_t i = 0; i < u; i++) {
    uint32_t below = bk_count_below(&b, x[i].rank);
    bk_insert(&b, x[i].rank);
    if (below < k) x[o++] = x[i];
  }
  return o;
}

/* Exported: prune an array of m entries given as parallel arrays; returns the
 * surviving count and rewrites the arrays in (distance, id) order. */
uint32_t orc_prune(uint64_t *d, uint32_t *id, uint32_t *rank, uint32_t m, uint32_t k) {
  ent *x = (ent *)malloc((size_t)(m ? m : 1) * sizeof(ent));
  uint32_t *bk = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  for (uint32_t i = 0; i < m; i++) { x[i].d = d[i]; x[i].id = id[i]; x[i].rank = rank[i]; }
  uint32_t o = prune_inplace(x, m, k, bk);
  for (uint32_t i = 0; i < o; i++) { d[i] = x[i].d; id[i] = x[i].id; rank[i] = x[i].rank; }
  free(x); free(bk);
  return o;
}

/* (iii) Alg. 2 as synchronous supersteps.  Each vertex receives the entries
 * its in-neighbours changed in the previous superstep, shifted by the arc
 * weight; it merges them into its sketch and runs CleanUp on the whole sketch
 * (the per-distance bottom-k rule, applied every superstep here), then sends
 * the entries that are new or got shorter.  Stops when no vertex sends. */
int orc_ads_rounds(const orc_graph *g, const uint32_t *rank, uint32_t k, orc_sketch *out,
                   uint32_t *n_rounds) {
  uint32_t n = g->n;
  entvec *sk = (entvec *)calloc(n, sizeof(entvec));
  entvec *delta = (entvec *)calloc(n, sizeof(entvec));
  entvec *ndelta = (entvec *)calloc(n, sizeof(entvec));
  uint32_t *bk = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  orc_rev rv; /* a vertex receives along its in-arcs */
  if (!sk || !delta || !ndelta || !bk || reverse_graph(g, &rv)) return ORC_ENOMEM;
  const orc_graph *gin = &rv.g;
  int rc = ORC_OK;
  for (uint32_t v = 0; v < n; v++) {
    ent e = {0, v, rank[v]};
    if (!ev_push(&sk[v], e) || !ev_push(&delta[v], e)) return ORC_ENOMEM;
  }
  uint32_t rounds = 0;
  entvec buf = {0};
  for (;;) {
    int any = 0;
    for (uint32_t v = 0; v < n; v++) if (delta[v].n) { any = 1; break; }
    if (!any) break;
    rounds++;
    for (uint32_t u = 0; u < n && rc == ORC_OK; u++) {
      buf.n = 0;
      int got = 0;
      for (uint64_t i = gin->row_ptr[u]; i < gin->row_ptr[u + 1]; i++) {
        uint32_t v = gin->col[i];
        for (uint32_t j = 0; j < delta[v].n; j++) {
          ent e = delta[v].a[j];
          e.d += arcw(gin, i);
          if (!ev_push(&buf, e)) { rc = ORC_ENOMEM; break; }
          got = 1;
        }
      }
      ndelta[u].n = 0;
      if (!got) continue;
      for (uint32_t j = 0; j < sk[u].n; j++)
        if (!ev_push(&buf, sk[u].a[j])) { rc = ORC_ENOMEM; break; }
      uint32_t m = prune_inplace(buf.a, buf.n, k, bk);
      /* entries that are new or shorter than before */
      for (uint32_t i = 0; i < m; i++) {
        int seen = 0;
        for (uint32_t j = 0; j < sk[u].n; j++)
          if (sk[u].a[j].id == buf.a[i].id && sk[u].a[j].d == buf.a[i].d) { seen = 1; break; }
        if (!seen && !ev_push(&ndelta[u], buf.a[i])) { rc = ORC_ENOMEM; break; }
      }
      /* the new sketch is stored in place after every vertex has read the old
       * deltas; sketches are private, so it can be written now */
      sk[u].n = 0;
      for (uint32_t i = 0; i < m; i++) ev_push(&sk[u], buf.a[i]);
    }
    entvec *tmp = delta; delta = ndelta; ndelta = tmp;
    if (rc != ORC_OK) break;
  }
  if (n_rounds) *n_rounds = rounds;
  if (rc == ORC_OK) rc = sketch_from_vecs(n, sk, out);
  for (uint32_t v = 0; v < n; v++) { free(sk[v].a); free(delta[v].a); free(ndelta[v].a); }
  free(sk); free(delta); free(ndelta); free(bk); free(buf.a);
  reverse_free(&rv);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* HIP-estimator weights (Sec. 3.3 names the estimator and its predicated use; */
/* the formula is the one of the cited ADS paper).  For entry j of a sketch in */
/* (distance, id) order, T_j is the k-th smallest rank among entries 0..j-1,   */
/* or 2^32 when j < k; the entry's weight is a_j = 2^32 / T_j (the inverse of  */
/* its inclusion probability with ranks read as uniform 32-bit values).        */
/* ------------------------------------------------------------------------ */
int orc_hipest(const orc_sketch *s, uint32_t n, uint32_t k, uint64_t *T, double *a) {
  uint32_t *bkv = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  if (!bkv) return ORC_ENOMEM;
  for (uint32_t v = 0; v < n; v++) {
    bottomk b = {bkv, 0, k};
    for (uint64_t j = s->off[v]; j < s->off[v + 1]; j++) {
      uint64_t Tj = b.n < k ? 4294967296ull : (uint64_t)b.v[k - 1];
      if (T) T[j] = Tj;
      if (a) a[j] = 4294967296.0 / (double)Tj;
      bk_insert(&b, s->rank[j]);
    }
  }
  free(bkv);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Facility location.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint8_t *open;         /* [n] 1 iff the vertex is in the returned set S */
  uint32_t *assign;      /* [n] nearest facility of S (ties: smaller id), ORC_NONE otherwise */
  uint32_t *dist;        /* [n] d(c, S) for served clients, ORC_NONE otherwise */
  uint32_t *open_rung;   /* [n] rung at which a facility opened (RUNG_*) */
  uint32_t *freeze_rung; /* [n] rung at which a client froze (RUNG_*) */
  double *q;             /* [n] final q(f) (0 for non-facilities) */
  uint64_t total_cost;
  uint32_t n_open, n_unreachable, n_rungs, mis_rounds, n_guard;
  uint64_t relax_alg, ads_entries, gamma;
  double alpha0, one_eps;
  uint32_t n_reach_guard; /* facilities added by the reach guard (directed graphs) */
} orc_result;

/* a[t] ladder (Sec. 4.2: alpha takes values alpha_0 (1+eps)^j); grown on demand */
typedef struct { double *a; uint32_t n, cap; double one_eps; } ladder;

static double lad_get(ladder *L, uint32_t t) {
  while (L->n <= t) {
    if (L->n == L->cap) {
      uint32_t nc = L->cap ? 2 * L->cap : 1024;
      double *na = (double *)realloc(L->a, (size_t)nc * sizeof(double));
      if (!na) return NAN;
      L->a = na; L->cap = nc;
    }
    L->a[L->n] = L->a[L->n - 1] * L->one_eps;
    L->n++;
  }
  return L->a[t];
}

/* bucket of a distance: the smallest ladder value that is >= d.  Reading: the
 * lowest bucket is [0, a[0]], so distance 0 (a facility that is also a
 * client) is counted. */
static double lad_beta(ladder *L, uint64_t d) {
  uint32_t j = 0;
  while (!((double)d <= lad_get(L, j))) j++;
  return L->a[j];
}

/* exact value a * 2^52 of a weight a >= 1 (every such double is a multiple of 2^-52) */
static __int128 fixed52(double a) { return (__int128)ldexp(a, 52); }

/* Bounded search: all vertices within distance <= rho (as doubles) of s,
 * along the given rows (on the reversed graph: all c with d(c, s) <= rho). */
static int ball(const orc_graph *g, uint32_t s, double rho, uint64_t *dist, uint32_t *list, uint32_t *cnt) {
  heap h = {0};
  uint32_t m = 0;
  dist[s] = 0;
  list[m++] = s;
  if (!hpush(&h, 0, s, s)) return ORC_ENOMEM;
  uint32_t nout = 0;
  uint32_t *out = (uint32_t *)malloc((size_t)g->n * sizeof(uint32_t));
  if (!out) return ORC_ENOMEM;
  while (h.n) {
    hitem it = hpop(&h);
    if (it.key != dist[it.v]) continue;
    out[nout++] = it.v;
    for (uint64_t i = g->row_ptr[it.v]; i < g->row_ptr[it.v + 1]; i++) {
      uint32_t y = g->col[i];
      uint64_t nd = it.key + arcw(g, i);
      if (!((double)nd <= rho)) continue;
      if (nd < dist[y]) {
        if (dist[y] == ORC_INF64) list[m++] = y;
        dist[y] = nd;
        if (!hpush(&h, nd, y, y)) { free(h.a); free(out); return ORC_ENOMEM; }
      }
    }
  }
  /* list holds every touched vertex (to reset dist); out the settled ones */
  for (uint32_t i = 0; i < m; i++) dist[list[i]] = ORC_INF64;
  memcpy(list, out, (size_t)nout * sizeof(uint32_t));
  *cnt = nout;
  free(out); free(h.a);
  return ORC_OK;
}

/* Luby's variant of the MIS (the baseline of Sec. 5.4): the same rounds, but
 * round r of a rung (r = 1, 2, ...) draws fresh priorities, a bijection keyed
 * by SplitMix64(seed ^ (3 + 256 r)). */
static uint64_t luby_key(uint64_t seed, uint32_t r) { return orc_splitmix64(seed ^ (3ull + 256ull * r)); }

static int solve_impl(const orc_graph *g, uint32_t k, uint64_t seed, double eps, int luby, orc_result *r);

int orc_solve(const orc_graph *g, uint32_t k, uint64_t seed, double eps, orc_result *r) {
  return solve_impl(g, k, seed, eps, 0, r);
}
int orc_solve_luby(const orc_graph *g, uint32_t k, uint64_t seed, double eps, orc_result *r) {
  return solve_impl(g, k, seed, eps, 1, r);
}

static int solve_impl(const orc_graph *g, uint32_t k, uint64_t seed, double eps, int luby, orc_result *r) {
  int rc = orc_validate(g, k, eps);
  if (r) r->n_open = 0;
  if (rc != ORC_OK) return rc;
  if (!g->fac_cost) return ORC_EINVAL;
  const uint32_t n = g->n;
  uint32_t *rank = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint32_t *prio = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!rank || !prio) return ORC_ENOMEM;
  orc_ranks(n, seed, rank, prio);
  /* distances from clients to facilities, d(c, f), come from searches that
   * start at facilities and follow the arcs backwards */
  orc_rev rv;
  if (reverse_graph(g, &rv)) return ORC_ENOMEM;
  const orc_graph *gb = &rv.g;

  /* Phase (i): neighbourhood sketching */
  orc_sketch sk = {0};
  rc = orc_ads_pruned(g, rank, k, &sk);
  if (rc != ORC_OK) return rc;
  uint64_t total = sk.off[n];
  double *aw = (double *)malloc((size_t)(total ? total : 1) * sizeof(double));
  if (!aw) return ORC_ENOMEM;
  orc_hipest(&sk, n, k, NULL, aw);
  r->ads_entries = total;
  r->relax_alg = 0;
  /* every entry of v is sent once along each arc out of v */
  for (uint32_t v = 0; v < n; v++)
    r->relax_alg += (sk.off[v + 1] - sk.off[v]) * (g->row_ptr[v + 1] - g->row_ptr[v]);

  /* gamma (Sec. 4.1): gamma_c = min_f c(f) + d(c,f); gamma = max over clients.
   * The same search records the minimising facility (ties: smaller id), used
   * only by the stall guard below. */
  uint64_t *ival = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *itie = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint64_t *gam = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *fstar = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  uint8_t *isF = (uint8_t *)calloc(n, 1), *isC = (uint8_t *)calloc(n, 1), *inU = (uint8_t *)calloc(n, 1);
  uint8_t *inO = (uint8_t *)calloc(n, 1), *inS = (uint8_t *)calloc(n, 1);
  uint64_t *dO = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *tmpt = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!ival || !itie || !gam || !fstar || !isF || !isC || !inU || !inO || !inS || !dO || !tmpt)
    return ORC_ENOMEM;
  uint32_t nF = 0, nC = 0;
  for (uint32_t v = 0; v < n; v++) {
    isF[v] = g->fac_cost[v] != NOT_FACILITY;
    isC[v] = g->is_client ? (g->is_client[v] != 0) : 1;
    nF += isF[v];
    ival[v] = isF[v] ? (uint64_t)g->fac_cost[v] : ORC_INF64;
    itie[v] = v;
    r->open_rung[v] = RUNG_NONE;
    r->freeze_rung[v] = RUNG_NONE;
    r->q[v] = 0.0;
    r->open[v] = 0;
    r->assign[v] = ORC_NONE;
    r->dist[v] = ORC_NONE;
  }
  rc = msdijkstra(gb, ival, itie, gam, fstar);
  if (rc != ORC_OK) return rc;
  uint64_t gamma = 0;
  uint32_t nU = 0, unreach = 0;
  for (uint32_t v = 0; v < n; v++) {
    if (!isC[v]) continue;
    nC++;
    if (gam[v] == ORC_INF64) { unreach++; continue; }
    inU[v] = 1; /* C_eff: clients that can reach a facility (reading: the
                   others are reported and left out of everything after) */
    nU++;
    if (gam[v] > gamma) gamma = gam[v];
  }
  r->gamma = gamma;
  r->n_unreachable = unreach;
  const uint32_t nCeff = nU;

  /* ladder: alpha_0 = gamma / m^2 * (1+eps) with m = |F| |C_eff| (Sec. 4.1) */
  ladder L = {0};
  L.one_eps = 1.0 + eps;
  r->one_eps = L.one_eps;
  r->alpha0 = 0.0;
  if (nF > 0 && nCeff > 0) {
    double M = (double)((uint64_t)nF * (uint64_t)nCeff);
    L.cap = 1024;
    L.a = (double *)malloc(1024 * sizeof(double));
    if (!L.a) return ORC_ENOMEM;
    L.a[0] = ((double)gamma / (M * M)) * L.one_eps;
    L.n = 1;
    r->alpha0 = L.a[0];
  }

  /* Opening phase: Alg. 4's sequential loop with Alg. 5 inside. */
  uint32_t nO = 0, t = 0, nguard = 0;
  for (uint32_t v = 0; v < n; v++) dO[v] = ORC_INF64;
  uint32_t *cursor = (uint32_t *)calloc(n, sizeof(uint32_t)); /* unused bookkeeping */
  uint32_t *newly = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!cursor || !newly) return ORC_ENOMEM;
  while (nO < nF && nU > 0) {
    /* Stall guard (not in the paper; never fires when every facility is a
     * reachable client).  Stuck iff no unopened facility has an unfrozen
     * client anywhere in its sketch and no unfrozen client has an open
     * facility at finite distance: then each such client opens its gamma
     * minimiser, which goes straight into S. */
    int live = 0;
    for (uint32_t f = 0; f < n && !live; f++) {
      if (!isF[f] || inO[f]) continue;
      for (uint64_t j = sk.off[f]; j < sk.off[f + 1]; j++)
        if (inU[sk.id[j]]) { live = 1; break; }
    }
    for (uint32_t c = 0; c < n && !live; c++)
      if (inU[c] && dO[c] != ORC_INF64) live = 1;
    if (!live) {
      for (uint32_t c = 0; c < n; c++) {
        if (!inU[c]) continue;
        uint32_t f = fstar[c];
        if (r->open_rung[f] != RUNG_GUARD) { r->open_rung[f] = RUNG_GUARD; nguard++; }
        r->freeze_rung[c] = RUNG_GUARD;
        inU[c] = 0;
        nU--;
      }
      break;
    }

    t++;
    double alpha = lad_get(&L, t); /* alpha grows before it is used (Alg. 4) */
    if (!isfinite(alpha)) return ORC_ERANGE;
    uint32_t nnew = 0;
    /* inU is not modified until the freeze step below, so it is the snapshot
     * of U visible to every facility in this rung */
    for (uint32_t f = 0; f < n; f++) {
      if (!isF[f] || inO[f]) continue;
      double inc;
      if (t == 1) {
        /* Eq. 2, read as the first evaluated rung: sum over sampled unfrozen
         * clients within alpha of a_j ((1+eps) alpha - beta(d_j)), in sketch
         * order */
        double ae = L.one_eps * alpha;
        inc = 0.0;
        for (uint64_t j = sk.off[f]; j < sk.off[f + 1]; j++) {
          if (!((double)sk.dist[j] <= alpha)) break;
          if (!inU[sk.id[j]]) continue;
          double b = lad_beta(&L, sk.dist[j]);
          inc = inc + aw[j] * (ae - b);
        }
      } else {
        /* Eq. 3: for buckets d <= alpha, max{0,(1+eps)alpha-d} - max{0,alpha-d}
         * = eps alpha, so t = eps alpha N(f, alpha) with N the HIP estimate of
         * unfrozen clients within alpha (predicated query), summed exactly */
        __int128 S = 0;
        for (uint64_t j = sk.off[f]; j < sk.off[f + 1]; j++) {
          if (!((double)sk.dist[j] <= alpha)) break;
          if (inU[sk.id[j]]) S += fixed52(aw[j]);
        }
        double Nhat = ldexp((double)S, -52);
        inc = (eps * alpha) * Nhat;
      }
      r->q[f] = r->q[f] + inc;
      if (r->q[f] >= (double)g->fac_cost[f]) newly[nnew++] = f;
    }
    for (uint32_t i = 0; i < nnew; i++) {
      inO[newly[i]] = 1;
      r->open_rung[newly[i]] = t;
      nO++;
    }
    if (nnew) {
      for (uint32_t v = 0; v < n; v++) { ival[v] = inO[v] ? 0 : ORC_INF64; itie[v] = 0; }
      rc = msdijkstra(gb, ival, itie, dO, tmpt);
      if (rc != ORC_OK) return rc;
    }
    /* Freeze (reading: Alg. 3's rule -- any open facility within
     * (1+eps) alpha(c), which is also the H-graph radius) */
    double rho = L.one_eps * alpha;
    for (uint32_t c = 0; c < n; c++) {
      if (!inU[c]) continue;
      if (dO[c] != ORC_INF64 && (double)dO[c] <= rho) {
        inU[c] = 0;
        nU--;
        r->freeze_rung[c] = t;
      }
    }
  }
  r->n_rungs = t;
  /* End phase: all facilities open, some clients unfrozen; they are tied to
   * their nearest facility and take part in no conflict (rung END). */
  if (nO == nF && nU > 0) {
    for (uint32_t c = 0; c < n; c++)
      if (inU[c]) { r->freeze_rung[c] = RUNG_END; inU[c] = 0; }
    nU = 0;
  }
  r->n_guard = nguard;

  /* MIS on H-bar, per rung (Sec. 4.3).  H edges join a client frozen at rung t
   * and a facility opened at rung t within (1+eps) a[t]; two facilities
   * conflict when they share such a client.  S_t is the greedy MIS taken in
   * increasing priority order (the result of the fixed-priority parallel
   * rounds); the rounds are also simulated to report their count and to check
   * that they give the same set. */
  uint64_t *bdist = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  uint32_t *blist = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!bdist || !blist) return ORC_ENOMEM;
  for (uint32_t v = 0; v < n; v++) bdist[v] = ORC_INF64;
  uint32_t mis_rounds = 0;
  /* facilities of each rung, listed by rung */
  uint32_t maxrung = t;
  uint32_t *rcount = (uint32_t *)calloc((size_t)maxrung + 2, sizeof(uint32_t));
  if (!rcount) return ORC_ENOMEM;
  for (uint32_t f = 0; f < n; f++)
    if (isF[f] && r->open_rung[f] >= 1 && r->open_rung[f] <= maxrung) rcount[r->open_rung[f]]++;
  for (uint32_t tt = 1; tt <= maxrung; tt++) {
    if (!rcount[tt]) continue;
    uint32_t m = rcount[tt];
    uint32_t *fac = (uint32_t *)malloc((size_t)m * sizeof(uint32_t));
    uint32_t mi = 0;
    for (uint32_t f = 0; f < n; f++)
      if (isF[f] && r->open_rung[f] == tt) fac[mi++] = f;
    /* sort facilities by priority (insertion sort; m is small in tests) */
    for (uint32_t i = 1; i < m; i++) {
      uint32_t x = fac[i], j = i;
      while (j > 0 && prio[fac[j - 1]] > prio[x]) { fac[j] = fac[j - 1]; j--; }
      fac[j] = x;
    }
    double rho = L.one_eps * lad_get(&L, tt);
    /* client lists: for each facility index i, its H_t clients */
    uint32_t **cl = (uint32_t **)calloc(m, sizeof(uint32_t *));
    uint32_t *ncl = (uint32_t *)calloc(m, sizeof(uint32_t));
    for (uint32_t i = 0; i < m; i++) {
      uint32_t cnt;
      rc = ball(gb, fac[i], rho, bdist, blist, &cnt); /* d(c, f) <= rho */
      if (rc != ORC_OK) return rc;
      cl[i] = (uint32_t *)malloc((size_t)(cnt ? cnt : 1) * sizeof(uint32_t));
      for (uint32_t z = 0; z < cnt; z++)
        if (isC[blist[z]] && r->freeze_rung[blist[z]] == tt) cl[i][ncl[i]++] = blist[z];
    }
    /* conflict test between facility indices i and j: a common client */
    uint8_t *adj = (uint8_t *)calloc((size_t)m * m, 1);
    {
      /* mark clients with their facility lists via a per-client scan */
      uint32_t *mark = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
      for (uint32_t v = 0; v < n; v++) mark[v] = ORC_NONE;
      for (uint32_t i = 0; i < m; i++) {
        for (uint32_t z = 0; z < ncl[i]; z++) mark[cl[i][z]] = i;
        for (uint32_t j = i + 1; j < m; j++)
          for (uint32_t z = 0; z < ncl[j]; z++)
            if (mark[cl[j][z]] == i) { adj[(size_t)i * m + j] = adj[(size_t)j * m + i] = 1; break; }
        for (uint32_t z = 0; z < ncl[i]; z++) mark[cl[i][z]] = ORC_NONE;
      }
      free(mark);
    }
    /* sequential greedy in priority order */
    uint8_t *gsel = (uint8_t *)calloc(m, 1);
    for (uint32_t i = 0; i < m; i++) {
      int ok = 1;
      for (uint32_t j = 0; j < i && ok; j++)
        if (gsel[j] && adj[(size_t)i * m + j]) ok = 0;
      gsel[i] = (uint8_t)ok;
    }
    /* parallel rounds: an active facility joins when no active neighbour
     * has a smaller priority (this round's priority for Luby's variant);
     * joined facilities retire their neighbours */
    uint8_t *act = (uint8_t *)malloc(m), *psel = (uint8_t *)calloc(m, 1), *join = (uint8_t *)malloc(m);
    uint32_t *pr = (uint32_t *)malloc((size_t)m * sizeof(uint32_t));
    memset(act, 1, m);
    uint32_t nact = m, rounds = 0;
    while (nact) {
      rounds++;
      for (uint32_t i = 0; i < m; i++)
        pr[i] = luby ? orc_perm(fac[i], luby_key(seed, rounds)) : prio[fac[i]];
      for (uint32_t i = 0; i < m; i++) {
        join[i] = 0;
        if (!act[i]) continue;
        int mn = 1;
        for (uint32_t j = 0; j < m && mn; j++)
          if (j != i && act[j] && adj[(size_t)i * m + j] && pr[j] < pr[i]) mn = 0;
        join[i] = (uint8_t)mn;
      }
      for (uint32_t i = 0; i < m; i++)
        if (join[i]) { psel[i] = 1; act[i] = 0; nact--; }
      for (uint32_t i = 0; i < m; i++) {
        if (!act[i]) continue;
        for (uint32_t j = 0; j < m; j++)
          if (join[j] && adj[(size_t)i * m + j]) { act[i] = 0; nact--; break; }
      }
    }
    mis_rounds += rounds;
    for (uint32_t i = 0; i < m; i++) {
      /* fixed priorities: the rounds give the greedy set (checked) */
      if (!luby && gsel[i] != psel[i]) return ORC_EINTERNAL;
      if (psel[i]) inS[fac[i]] = 1;
    }
    for (uint32_t i = 0; i < m; i++) free(cl[i]);
    free(cl); free(ncl); free(adj); free(gsel); free(act); free(psel); free(join); free(fac); free(pr);
  }
  r->mis_rounds = mis_rounds;
  for (uint32_t f = 0; f < n; f++)
    if (isF[f] && r->open_rung[f] == RUNG_GUARD) inS[f] = 1;

  /* Reach guard (not in the paper; never fires on an undirected graph, where
   * a client reaches every facility of its component).  On a directed graph
   * a client's facility can lose the MIS to a conflicting one the client
   * cannot reach.  Every served client that reaches no facility of S opens
   * its gamma minimiser, which it reaches by definition, straight into S. */
  r->n_reach_guard = 0;
  for (uint32_t v = 0; v < n; v++) { ival[v] = inS[v] ? 0 : ORC_INF64; itie[v] = v; }
  rc = msdijkstra(gb, ival, itie, dO, tmpt);
  if (rc != ORC_OK) return rc;
  for (uint32_t c = 0; c < n; c++) {
    if (!isC[c] || gam[c] == ORC_INF64 || dO[c] != ORC_INF64) continue;
    if (!inS[fstar[c]]) { inS[fstar[c]] = 1; r->n_reach_guard++; }
  }

  /* Assignment and objective (Sec. 3.1): each served client goes to its
   * nearest facility of S (ties: smaller id); cost = sum of opening costs of
   * S plus the sum of client distances. */
  for (uint32_t v = 0; v < n; v++) { ival[v] = inS[v] ? 0 : ORC_INF64; itie[v] = v; }
  rc = msdijkstra(gb, ival, itie, dO, tmpt);
  if (rc != ORC_OK) return rc;
  uint64_t cost = 0;
  uint32_t nopen = 0;
  for (uint32_t v = 0; v < n; v++) {
    if (inS[v]) { r->open[v] = 1; nopen++; cost += g->fac_cost[v]; }
  }
  for (uint32_t v = 0; v < n; v++) {
    if (!isC[v] || gam[v] == ORC_INF64) continue;
    if (dO[v] == ORC_INF64) return ORC_EINTERNAL; /* a served client always reaches S */
    r->assign[v] = tmpt[v];
    r->dist[v] = (uint32_t)dO[v];
    cost += dO[v];
  }
  r->total_cost = cost;
  r->n_open = nopen;

  orc_sketch_free(&sk);
  free(aw); free(rank); free(prio); free(ival); free(itie); free(gam); free(fstar);
  free(isF); free(isC); free(inU); free(inO); free(inS); free(dO); free(tmpt);
  free(cursor); free(newly); free(bdist); free(blist); free(rcount); free(L.a);
  reverse_free(&rv);
  return ORC_OK;
}

/* Ladder values as the solve computes them (for closed-form checks). */
int orc_ladder(double alpha0, double eps, uint32_t count, double *out) {
  if (count == 0) return ORC_OK;
  double one_eps = 1.0 + eps;
  out[0] = alpha0;
  for (uint32_t t = 1; t < count; t++) out[t] = out[t - 1] * one_eps;
  return ORC_OK;
}

/* Exhaustive optimum over all non-empty facility subsets (|F| <= 20):
 * min over S of sum_{f in S} c(f) + sum_{c in C_eff} d(c, S); subsets that
 * leave a served client at infinite distance are skipped. */
int orc_opt_exhaustive(const orc_graph *g, uint64_t *best_cost) {
  uint32_t n = g->n;
  uint32_t F[20], nF = 0;
  for (uint32_t v = 0; v < n; v++)
    if (g->fac_cost[v] != NOT_FACILITY) {
      if (nF == 20) return ORC_EINVAL;
      F[nF++] = v;
    }
  if (nF == 0) { *best_cost = 0; return ORC_OK; }
  uint64_t *D = (uint64_t *)malloc((size_t)nF * n * sizeof(uint64_t));
  orc_rev rv;
  if (!D || reverse_graph(g, &rv)) return ORC_ENOMEM;
  /* D[i][c] = d(c, F[i]) */
  for (uint32_t i = 0; i < nF; i++) dijkstra(&rv.g, F[i], D + (size_t)i * n, NULL, NULL);
  uint64_t best = ORC_INF64;
  for (uint64_t mask = 1; mask < (1ull << nF); mask++) {
    uint64_t cost = 0;
    int ok = 1;
    for (uint32_t i = 0; i < nF; i++)
      if (mask >> i & 1) cost += g->fac_cost[F[i]];
    for (uint32_t c = 0; c < n && ok; c++) {
      int client = g->is_client ? g->is_client[c] != 0 : 1;
      if (!client) continue;
      uint64_t anyd = ORC_INF64, d = ORC_INF64;
      for (uint32_t i = 0; i < nF; i++) {
        uint64_t x = D[(size_t)i * n + c];
        if (x < anyd) anyd = x;
        if ((mask >> i & 1) && x < d) d = x;
      }
      if (anyd == ORC_INF64) continue; /* unreachable client: not served */
      if (d == ORC_INF64) ok = 0;
      else cost += d;
    }
    if (ok && cost < best) best = cost;
  }
  free(D);
  reverse_free(&rv);
  *best_cost = best;
  return ORC_OK;
}
