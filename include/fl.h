/*
 * fl.h -- C ABI of the MI355X (gfx950) library for sketch-based facility
 * location on graphs, after "Scalable Facility Location for Massive Graphs on
 * Pregel-like Systems" (arXiv 1503.03635).
 *
 * Problem (Sec. 3.1 of the paper): an undirected graph G = (V, E, w), a set of
 * facilities F with opening costs c(f), a set of clients C, distances d given
 * by shortest paths in G.  Pick S subset of F minimising
 *     sum_{f in S} c(f) + sum_{c in C} d(c, S).
 * Method (Sec. 3.3 and Sec. 4): bottom-k all-distances sketches (ADS) for
 * every vertex, the opening loop of Alg. 4/Alg. 5 driven by HIP-estimator
 * neighbourhood estimates (Eq. 2, Eq. 3), freezing of clients near open
 * facilities, and a maximal independent set on the conflict graph H-bar
 * (Sec. 4.3, Alg. 6) to pick S.
 *
 * Conventions for every call below
 *   - Every array in fl_problem and fl_result is a DEVICE pointer (memory of
 *     the current HIP device, e.g. a torch tensor's data_ptr()).  The caller
 *     owns all of them; the library never frees or modifies inputs.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it; the call synchronises it before it
 *     returns host scalars, so device outputs are valid on return.
 *   - Return value: FL_OK (0) or one of the FL_E* codes.  On error the device
 *     outputs are unspecified and result->n_open is 0.
 *   - The library keeps a per-device workspace cache between calls (released
 *     by fl_release_workspace).  Calls that overlap on one device from
 *     several host threads are serialised internally.
 *
 * Environment (read at each call; neither changes any result)
 *   - FL_DEBUG: progress lines of the sketch rounds and the workspace
 *     allocations on stderr, and extra sketch-round counters.
 *   - FL_TEST_SMALL_SURVIVOR_BUFFER: test hook.  Sketch builds with k <= 64
 *     start with the small survivor buffer that k <= 32 uses (512 ids per
 *     level), so that modest inputs reach the restart with the full buffer.
 */
#ifndef FL_H_
#define FL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define FL_OK 0
#define FL_EINVAL 1   /* malformed/asymmetric CSR, unsorted or duplicate neighbours,
                         self loop, w = 0, k = 0, eps <= 0 or not finite,
                         n = 0 or n >= 2^32-1, NULL required pointer */
#define FL_ERANGE 2   /* (n-1)*max(w) + max(c) >= 2^32-1: a distance or a cost
                         plus distance could overflow 32 bits */
#define FL_ENOMEM 3   /* workspace does not fit the device (or the budget) */
#define FL_EHIP 4     /* a HIP runtime error; see fl_last_hip_error() */
#define FL_EBUSY 5    /* server queue full (non-blocking submit) */
#define FL_ENOTIMPL 6 /* a limit of this library: k > 128, max weight > 255,
                         sketch capacity above 65535 entries per vertex */

/* ---- sentinels ---------------------------------------------------------- */
#define FL_NOT_FACILITY 0xFFFFFFFFu /* fac_cost value of a non-facility vertex */
#define FL_NONE 0xFFFFFFFFu         /* assign/dist of a non-client or unreachable client */
#define FL_RUNG_NONE 0xFFFFFFFFu    /* never opened / never frozen */
#define FL_RUNG_GUARD 0xFFFFFFFEu   /* opened or frozen by the stall guard */
#define FL_RUNG_END 0xFFFFFFFDu     /* frozen in the end phase (all facilities open) */

/* ---- problem: graph in symmetric CSR, costs, clients (Sec. 3.1) ---------- */
/* With FL_FLAG_DIRECTED the rows are out-arcs and the symmetry rules below
 * do not apply; every other rule does. */
typedef struct {
  uint32_t n;               /* |V|, 1 <= n < 2^32-1 */
  uint64_t n_arcs;          /* 2|E| (directed: the number of arcs) */
  const uint64_t *row_ptr;  /* [n+1], row_ptr[0] = 0, row_ptr[n] = n_arcs */
  const uint32_t *col;      /* [n_arcs], strictly increasing within each row,
                               no self loops; (u,v) present iff (v,u) present */
  const uint32_t *w;        /* [n_arcs] integer weights >= 1, equal on (u,v) and
                               (v,u); NULL = unit weights */
  const uint32_t *fac_cost; /* [n] opening cost c(f); FL_NOT_FACILITY marks a
                               vertex that is not a facility.  Required by
                               fl_solve, ignored by fl_ads_build. */
  const uint8_t *is_client; /* [n] nonzero = client; NULL = every vertex */
} fl_problem;

/* ---- parameters ---------------------------------------------------------- */
typedef struct {
  uint32_t k;     /* bottom-k parameter of the sketches, 1 <= k <= 128 */
  uint64_t seed;  /* seeds the vertex ranks and the MIS priorities */
  double eps;     /* accuracy parameter epsilon > 0 (the paper's runs use 0.1) */
  uint32_t flags; /* FL_FLAG_* below */
} fl_params;

#define FL_FLAG_NO_DENSE 1u  /* always use frontier worklists in the ADS rounds */
#define FL_FLAG_LUBY_MIS 2u  /* Luby's MIS variant (the baseline the paper compares
                                against, Sec. 5.4): the same rounds as Alg. 6, but
                                round r of a rung draws fresh priorities, a
                                bijection of the local id keyed by
                                SplitMix64(seed ^ (3 + 256 r)).  A maximal
                                independent set, in general not the greedy one. */
#define FL_FLAG_DIRECTED 4u  /* the CSR holds the out-arcs of a directed graph
                                (Sec. 3.1 considers both kinds; Sec. 4.4: the
                                method carries over, without its guarantee).
                                No reverse arcs are required.  d(u, v) is then the
                                shortest path along arcs from u to v; the sketch
                                of v holds the vertices that reach v, at d(u, v)
                                (entries travel along arcs, Alg. 2); clients are
                                counted by, frozen by, in conflict through and
                                assigned to facilities they can reach, at d(c, f);
                                gamma and unreachable clients likewise.  On a
                                symmetric CSR the result equals the undirected
                                one.  Costs an in-arc copy of the graph in the
                                workspace (8(n+1) + 4 n_arcs bytes, 8 n_arcs when
                                weighted). */

/* ---- statistics ---------------------------------------------------------- */
typedef struct {
  uint32_t ads_rounds;  /* distance rounds of the sketch construction */
  uint32_t rungs;       /* radius-ladder rungs evaluated by the opening loop */
  uint32_t mis_rounds;  /* parallel MIS rounds, summed over rungs */
  uint32_t n_guard;     /* facilities opened by the stall guard */
  uint64_t relax_alg;   /* sum_v |ADS(v)| * deg(v) (directed: out-degree) */
  uint64_t relax_exec;  /* candidate entries read by the sketch rounds */
  uint64_t ads_entries; /* sum_v |ADS(v)| */
  uint64_t gamma;       /* max over served clients of min_f c(f) + d(c,f) */
  double alpha0;        /* first ladder value */
  double ms_validate, ms_ads, ms_gamma, ms_open, ms_mis, ms_assign, ms_total;
  double ms_ads_kernel;          /* summed device time of the sketch-round kernel launches
                                    (k_ads_tasks, one per distance round; rounds launched 16
                                    at a time also count the empty rounds that end their last
                                    chunk) */
  double ms_ads_merge;           /* summed device time of the merges of split hub vertices */
  uint32_t ads_kernel_launches;  /* number of sketch-round kernel launches */
  uint64_t workspace_bytes;
  uint32_t n_reach_guard;  /* facilities added because a served client reached no
                              facility of S (directed graphs only: each such client
                              opens its gamma minimiser, argmin_f c(f) + d(c,f),
                              ties by id); always 0 on an undirected graph */
} fl_stats;

/* ---- result -------------------------------------------------------------- */
typedef struct {
  /* caller-owned device outputs, each [n] */
  uint8_t *open;         /* 1 iff the vertex is in the returned set S */
  uint32_t *assign;      /* nearest facility of S (ties: smaller id) for every
                            served client; FL_NONE otherwise */
  uint32_t *dist;        /* d(c, S) for served clients, FL_NONE otherwise; may be NULL */
  uint32_t *open_rung;   /* optional (NULL): rung at which each facility opened */
  uint32_t *freeze_rung; /* optional (NULL): rung at which each client froze */
  double *q;             /* optional (NULL): final q(f) of each facility, 0 elsewhere */
  /* host scalars, written by the call */
  uint64_t total_cost;   /* sum_{f in S} c(f) + sum over served clients d(c, S) */
  uint32_t n_open;       /* |S| */
  uint32_t n_unreachable;/* clients with no facility in their component */
  int32_t status;        /* FL_OK or this element's error code (set by fl_solve
                            and by fl_solve_batch for every element) */
  fl_stats stats;
} fl_result;

/*
 * fl_solve -- one complete facility-location solve (Alg. 4 with Alg. 5 and
 * Alg. 6 inside): validate the CSR, build the bottom-k ADS of every vertex,
 * compute gamma and the radius ladder (Sec. 4.1-4.2), run the opening loop
 * with HIP-estimator estimates of the unfrozen clients near each facility,
 * resolve conflicts per rung with the fixed-priority MIS, assign clients and
 * add up the objective.  Clients that cannot reach any facility are reported
 * (FL_NONE, n_unreachable) and left out of the objective.
 */
int fl_solve(const fl_problem *p, const fl_params *prm, fl_result *out, void *stream);

/*
 * fl_solve_static -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same solve, arguments and results as fl_solve, but the
 * library's workspace is carved from one fixed device array of
 * FL_STATIC_SCRATCH_BYTES that every device loading the library holds until
 * the process ends.  The call allocates no device or pinned host memory and
 * creates no HIP events (the ms_* statistics stay 0); its host bookkeeping
 * uses the ordinary C++ heap.  The caller still passes every input and output.
 *   - FL_ENOMEM when the solve needs more than the array: at once, before any
 *     device work, when the sketch rows alone (n x capacity x 8 bytes, the
 *     capacity being about k (1 + ln(n/k)) entries plus a margin) do not
 *     fit; otherwise as soon as a further piece of the workspace would cross
 *     the array's end (no pointer past it is ever handed out).
 *   - Every call on a device uses that device's one array and finds the
 *     previous call's contents there; the solve initialises all it reads.
 *     Two calls whose device work overlapped on one device would race on the
 *     array, so calls on a device are serialised and each synchronises its
 *     stream before it returns.
 */
#define FL_STATIC_SCRATCH_BYTES (256ull << 20)
int fl_solve_static(const fl_problem *p, const fl_params *prm, fl_result *out, void *stream);

/*
 * fl_solve_batch -- `count` independent solves; per element the same contract
 * and the same results as fl_solve (its status field says whether it
 * succeeded).  Elements with equal k, eps and flags are solved together as one
 * disjoint union of their graphs: every phase (sketch rounds, opening rungs,
 * MIS sweeps, assignment) runs once for the whole group instead of once per
 * graph, with per-graph ranks, priorities, ladders and rung counters.  Groups
 * are cut to fit 60% of the device memory; the estimate uses each weighted
 * graph's largest weight, read by one launch over all elements before the
 * cut, so every element's w must hold n_arcs readable entries (as for
 * fl_solve).  Statistics that describe the whole group
 * (ads_rounds, relax_exec, the ms_* times, workspace_bytes) are reported for
 * every element of the group.  Returns FL_OK or the first element error.
 */
int fl_solve_batch(const fl_problem *ps, const fl_params *prms, fl_result *outs, uint32_t count,
                   void *stream);

/* ---- serving: continuous batching ------------------------------------------
 * A server solves requests as they arrive.  It owns `slots` workers on the
 * current device, each with its own stream and workspace.  A free worker takes
 * the oldest waiting request together with later waiting ones of equal k, eps
 * and flags, as many as fit the device-memory budget, and solves them as one
 * group (the disjoint union of fl_solve_batch).  Requests that arrive while
 * others are on the GPU wait until a worker and memory free up; work of
 * different workers overlaps on the device.  Every result equals fl_solve of
 * the same request alone.
 *
 * The caller keeps each request's problem, params and result (and the device
 * buffers they point to) alive until fl_server_poll reports it finished or
 * fl_server_wait returns for it.  The server keeps no pointer afterwards.
 */
typedef struct fl_server fl_server;

/* hbm_budget_bytes: device memory the workers' workspaces may hold together
 * (0 = 60% of the free memory); slots: workers (0 = 3).  FL_EINVAL if a
 * request alone can never fit is reported per request at submission. */
int fl_server_create(uint64_t hbm_budget_bytes, uint32_t slots, fl_server **out);
/* Queues one request; *ticket identifies it.  FL_EINVAL for bad arguments,
 * FL_ENOMEM if the request alone exceeds the budget, FL_EBUSY if the server is
 * shutting down. */
int fl_server_submit(fl_server *s, const fl_problem *p, const fl_params *prm, fl_result *out, uint64_t *ticket);
/* FL_OK with *status = the request's code when it has finished (the ticket is
 * then retired), FL_EBUSY while it is queued or running, FL_EINVAL for an
 * unknown ticket. */
int fl_server_poll(fl_server *s, uint64_t ticket, int *status);
/* Blocks until the request finishes; then as fl_server_poll. */
int fl_server_wait(fl_server *s, uint64_t ticket, int *status);
/* Finishes every queued and running request, then frees the server. */
void fl_server_destroy(fl_server *s);

/* ---- sketches (Sec. 3.3) --------------------------------------------------- */
typedef struct fl_sketch fl_sketch;

typedef struct {
  uint32_t n, k;
  uint64_t total;          /* sum_v |ADS(v)| */
  const uint64_t *off;     /* device [n+1]: entries of v are [off[v], off[v+1]) */
  const uint32_t *rank;    /* device [total]: rank of the sampled vertex */
  const uint32_t *dist;    /* device [total]: its distance from v */
  const uint32_t *thresh;  /* device [total]: HIP threshold T_j (k-th smallest rank
                              among earlier entries), 0 meaning 2^32 (j < k) */
} fl_sketch_view_t;

/*
 * fl_ads_build -- bottom-k ADS of every vertex.  Entry order within a vertex
 * is increasing (distance, vertex id); entry 0 is (r(v), 0).  The library
 * owns the storage until fl_sketch_free.  fac_cost is not read.
 */
int fl_ads_build(const fl_problem *p, const fl_params *prm, fl_sketch **out, void *stream);
/* Fills *view with device pointers into the sketch (valid until free). */
int fl_sketch_view(const fl_sketch *s, fl_sketch_view_t *view);
void fl_sketch_free(fl_sketch *s);

/* Vertex rank r(v) and MIS priority of the given seed (host helpers; the
 * library computes the same values on the device). */
uint32_t fl_rank_of(uint32_t v, uint64_t seed);
uint32_t fl_priority_of(uint32_t v, uint64_t seed);

/* ---- errors and resources -------------------------------------------------- */
const char *fl_strerror(int code);
int fl_last_hip_error(void);
/* Frees the cached workspace of the current device. */
void fl_release_workspace(void);

/* Device-memory hooks (optional; the library's own resources, not part of
 * the method).  With alloc set, every device allocation the library makes
 * (the cached per-device workspace, the batch and server workspaces, sketch
 * handles) goes through alloc(bytes, device, ctx) and later
 * free_fn(ptr, bytes, device, ctx) instead of hipMalloc/hipFree, e.g. so that
 * a framework's caching allocator backs it.  `device` is the HIP device that
 * is current for the call.  alloc returns NULL on failure (the call then
 * reports FL_ENOMEM); the memory must stay valid until free_fn is called and
 * be usable from any stream.  fl_set_allocator(NULL, NULL, NULL) restores
 * hipMalloc/hipFree.  Cached workspaces are released first, each through the
 * hooks it came from; a live sketch handle keeps its hooks until
 * fl_sketch_free.  Returns FL_EBUSY while a server exists, FL_EINVAL if only
 * one of alloc and free_fn is NULL, else FL_OK.  Not to be called while
 * another library call is running.  The hooks run inside library calls
 * (possibly on the server's worker threads) and must not call into this
 * library themselves. */
typedef void *(*fl_alloc_fn)(size_t bytes, int device, void *ctx);
typedef void (*fl_free_fn)(void *ptr, size_t bytes, int device, void *ctx);
int fl_set_allocator(fl_alloc_fn alloc, fl_free_fn free_fn, void *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FL_H_ */
