// fl_mis.hip -- facility selection: a maximal independent set of the
// conflict graph H-bar, per rung (Sec. 4.3, Alg. 6), without building H.
//
// A client c and a facility f are joined in H when both carry the same rung
// t (c froze at t, f opened at t) and d(c, f) <= (1 + eps) a[t]; facilities
// conflict when they share a client.  Priorities pi(f) are a seeded
// bijection, and each round of the fixed-priority algorithm is four bounded
// sweeps over the graph:
//   1. every client takes the smallest priority of the active facilities
//      within the radius (pi_min);
//   2. every active facility takes the smallest pi_min of the clients within
//      the radius; it joins S when that is its own priority (or when it has
//      no client);
//   3. clients within the radius of a joined facility are covered;
//   4. active facilities within the radius of a covered client retire.
// Rounds repeat until no facility is active; the result is the greedy MIS in
// priority order.  The radius is measured from client to facility, d(c, f):
// sweeps 1 and 3 start at facilities and push over the in-arcs, sweeps 2 and
// 4 start at clients and push over the out-arcs (the same arcs when the graph
// is undirected).  In a union of several graphs, each graph walks through its
// own non-empty rungs: step i runs the i-th one of every graph at once (the
// graphs share no vertex, so their sweeps do not interact), each with its own
// radius and priorities.  A sweep computes, for every vertex x, the minimum label
// over sources within distance R of x.  It runs in distance order (round j
// settles labels at distance exactly j) with one pending-label array per
// distance slot modulo max_w + 1, so a label is forwarded only when it
// lowers a vertex's current minimum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fl_common.h"
#include "fl_frontier.h"
#include "fl_mis.h"

namespace fl {

struct SweepArgs {
  uint32_t n, NS;
  const uint32_t *gid;  // graph of each vertex (nullptr: one graph)
  const uint32_t *Rg;   // [G] radius of each graph in the current step
  const uint64_t *row_ptr;
  const uint32_t *col;
  const uint32_t *w;
  uint32_t *ml;       // [n] current minimum label (INF32 = none)
  uint32_t *pend;     // [NS * n] pending label per slot
  uint32_t *tl;       // [NS * n] vertices with a pending label per slot
  uint32_t *tl_cnt;   // [NS * CNT_PAD] list length of each slot, one per line
  uint32_t *touched;  // [n] vertices whose ml was set
  uint32_t *touched_cnt;
  uint64_t *heavy;    // pieces of the long rows queued in the current distance
  uint32_t *heavy_cnt;  // [2] by distance parity
  const uint32_t *tbits;  // bitmap of the vertices whose result is read (nullptr: all)
};

// Queue appends (vertex y to the list of slot s), staged per wave in LDS
// (2 WAVE entries) and written WAVE at a time with one atomic per distinct
// slot among them: with per-step atomics the waves of a large frontier queue
// on the slot's one count.
struct SlotQ {
  uint32_t *ys, *ss;  // this wave's LDS staging: vertices and their slots
  uint32_t cnt;       // staged entries (wave-uniform, < WAVE between calls)
};

// append y to the list of slot s on the lanes with have set: one atomic per
// distinct slot among them
__device__ inline void slotq_write(const SweepArgs &S, bool have, uint32_t y, uint32_t s) {
  const int lane = lane_id();
  uint64_t pendm = __ballot(have);
  while (pendm) {
    const int lead = __ffsll((long long)pendm) - 1;
    const uint32_t sl = __shfl(s, lead, WAVE);
    const bool mine = have && s == sl;
    const uint64_t grp = __ballot(mine);
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(&S.tl_cnt[sl * CNT_PAD], (uint32_t)__popcll(grp));
    base = __shfl(base, lead, WAVE);
    if (mine) {
      S.tl[(size_t)sl * S.n + base + lanes_below(grp)] = y;
      have = false;
    }
    pendm &= ~grp;
  }
}

// every lane calls, converged
__device__ inline void slotq_push(const SweepArgs &S, SlotQ &q, bool add, uint32_t y, uint32_t s) {
  const int lane = lane_id();
  const uint64_t m = __ballot(add);
  if (!m) return;
  if (add) {
    q.ys[q.cnt + lanes_below(m)] = y;
    q.ss[q.cnt + lanes_below(m)] = s;
  }
  q.cnt += (uint32_t)__popcll(m);
  if (q.cnt < (uint32_t)WAVE) return;
  wave_lds_sync();
  slotq_write(S, true, q.ys[lane], q.ss[lane]);
  q.cnt -= WAVE;
  const bool more = (uint32_t)lane < q.cnt;
  const uint32_t ry = more ? q.ys[WAVE + lane] : 0u, rs = more ? q.ss[WAVE + lane] : 0u;
  wave_lds_sync();
  if (more) {
    q.ys[lane] = ry;
    q.ss[lane] = rs;
  }
  wave_lds_sync();
}

// the staged remainder (every lane calls, converged, before the wave exits)
__device__ inline void slotq_flush(const SweepArgs &S, SlotQ &q) {
  if (!q.cnt) return;
  const int lane = lane_id();
  wave_lds_sync();
  const bool have = (uint32_t)lane < q.cnt;
  slotq_write(S, have, have ? q.ys[lane] : 0u, have ? q.ss[lane] : 0u);
  q.cnt = 0;
}

// LDS staging for the 256 / WAVE waves of a block
#define SLOTQ_DECL(q)                                   \
  __shared__ uint32_t q##_ys[256 / WAVE][2 * WAVE];     \
  __shared__ uint32_t q##_ss[256 / WAVE][2 * WAVE];     \
  SlotQ q{q##_ys[threadIdx.x / WAVE], q##_ss[threadIdx.x / WAVE], 0u}

// Two arc steps of a push (every lane calls, converged; a lane with v0 or v1
// false has no arc in that group): per arc, lower the pending label of the
// head at distance j + w when that is within R, and queue the head once per
// slot.  Both groups' columns, weights and head minima are loaded before
// either group is tested, so a wave keeps two chains of dependent reads in
// flight instead of one (on the large weighted workload MIS went 1.17 ->
// 1.11 s from the long rows, then 1.106 -> 1.095 s from the short rows).
// A head whose settled minimum is already at most the label is skipped: it
// reached that minimum at a smaller distance, so the push could never settle
// (a concurrent settle only lowers ml, which keeps the test safe).  A label
// landing at distance exactly R goes no further, so there it is kept only at
// the sweep's targets, the vertices whose minimum is read afterwards.
__device__ inline void sweep_arcs2(const SweepArgs &S, SlotQ &q, uint32_t j, bool v0, uint64_t i0, uint32_t lab0,
                                   uint32_t R0, bool v1, uint64_t i1, uint32_t lab1, uint32_t R1) {
  const uint32_t y0 = v0 ? S.col[i0] : 0u, y1 = v1 ? S.col[i1] : 0u;
  const uint32_t w0 = v0 ? (S.w ? S.w[i0] : 1u) : 0u, w1 = v1 ? (S.w ? S.w[i1] : 1u) : 0u;
  const uint64_t d0 = (uint64_t)j + w0, d1 = (uint64_t)j + w1;
  const bool k0 = v0 && (d0 < R0 || (d0 == R0 && (!S.tbits || ((S.tbits[y0 >> 5] >> (y0 & 31)) & 1u))));
  const bool k1 = v1 && (d1 < R1 || (d1 == R1 && (!S.tbits || ((S.tbits[y1 >> 5] >> (y1 & 31)) & 1u))));
  const uint32_t m0 = k0 ? __hip_atomic_load(&S.ml[y0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
  const uint32_t m1 = k1 ? __hip_atomic_load(&S.ml[y1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
  bool add0 = false, add1 = false;
  uint32_t s0 = 0, s1 = 0;
  if (k0 && lab0 < m0) {
    s0 = (j + w0) % S.NS;
    uint32_t *p = &S.pend[(size_t)s0 * S.n + y0];
    if (lab0 < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) add0 = atomicMin(p, lab0) == INF32;
  }
  if (k1 && lab1 < m1) {
    s1 = (j + w1) % S.NS;
    uint32_t *p = &S.pend[(size_t)s1 * S.n + y1];
    if (lab1 < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) add1 = atomicMin(p, lab1) == INF32;
  }
  slotq_push(S, q, add0, y0, s0);
  slotq_push(S, q, add1, y1, s1);
}

// The short rows of the lanes flattened over the wave, two steps of 64 arcs
// per call of f(v0, arc0, owner0, v1, arc1, owner1) (every lane calls,
// converged): arc c*64 + lane of the concatenated rows is found by a binary
// search over the running degree sum, as in flat_arcs.
template <class F>
__device__ inline void flat_arcs2(bool light, uint64_t a0, uint64_t deg, F &&f) {
  const int lane = lane_id();
  const uint32_t d = light ? (uint32_t)deg : 0u;
  const uint32_t incl = wave_scan_incl(d);
  const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
  const uint32_t excl = incl - d;
  auto locate = [&](uint32_t idx, bool &valid, uint64_t &arc, int &own) {
    uint32_t pos = 0;  // first lane whose inclusive sum exceeds idx
#pragma unroll
    for (uint32_t s = 32; s >= 1; s >>= 1) {
      const uint32_t val = __shfl(incl, (int)(pos + s - 1), WAVE);
      if (val <= idx) pos += s;
    }
    valid = idx < total;
    own = valid ? (int)pos : 0;
    arc = shfl_u64(a0, own) + (idx - __shfl(excl, own, WAVE));
  };
  for (uint32_t c0 = 0; c0 < total; c0 += 2 * WAVE) {
    bool v0, v1;
    uint64_t x0, x1;
    int o0, o1;
    locate(c0 + (uint32_t)lane, v0, x0, o0);
    locate(c0 + WAVE + (uint32_t)lane, v1, x1, o1);
    f(v0, x0, o0, v1, x1, o1);
  }
}

// Rows of a sweep flattened over the wave: at most this many arcs (half the
// other frontier kernels' FLAT_MAX).  Longer rows go to k_sweep_heavy, whose
// waves keep more reads in flight than a flattened step: MIS 0.898 -> 0.835 s
// on the large weighted workload against 256, timed on one box, identical
// results.
constexpr uint32_t SWEEP_FLAT_MAX = 128;

// Push the labels of the lanes' vertices (want) from distance j: short rows
// flattened over the wave, long rows queued for k_sweep_heavy.
__device__ inline void sweep_push_lanes(const SweepArgs &S, SlotQ &q, bool want, uint32_t x, uint32_t lab,
                                        uint32_t j) {
  uint64_t a0 = 0, deg = 0;
  uint32_t R = 0;
  if (want) {
    R = S.Rg[seg_of(S.gid, x)];
    want = j < R;  // arcs weigh at least 1: a label settled at distance R goes no further
  }
  if (want) {
    a0 = S.row_ptr[x];
    deg = S.row_ptr[x + 1] - a0;
  }
  const bool heavy = want && deg > SWEEP_FLAT_MAX;
  push_pieces(S.heavy, S.heavy_cnt + (j & 1), heavy, x, deg);
  flat_arcs2(want && !heavy, a0, deg, [&](bool v0, uint64_t x0, int o0, bool v1, uint64_t x1, int o1) {
    sweep_arcs2(S, q, j, v0, x0, __shfl(lab, o0, WAVE), __shfl(R, o0, WAVE), v1, x1, __shfl(lab, o1, WAVE),
                __shfl(R, o1, WAVE));
  });
}

// vertices whose ml was set for the first time -> touched (one atomic per wave)
__device__ inline void touch(const SweepArgs &S, bool first, uint32_t x) {
  wave_push(S.touched, S.touched_cnt, first, x);
}

// sources: set ml and push at distance 0 (one lane per source)
__global__ __launch_bounds__(256) void k_sweep_init(SweepArgs S, const uint32_t *src, uint32_t nsrc,
                                                    const uint32_t *lab) {
  SLOTQ_DECL(q);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool want = false;
  uint32_t x = 0, l = INF32;
  if (i < nsrc) {
    x = src[i];
    l = lab[x];
    want = l != INF32;
    if (want) S.ml[x] = l;
  }
  touch(S, want, x);
  sweep_push_lanes(S, q, want, x, l, 0);
  slotq_flush(S, q);
}

// distance j: settle the pending labels of slot j (one lane per vertex)
__global__ __launch_bounds__(256) void k_sweep_round(SweepArgs S, uint32_t j) {
  SLOTQ_DECL(q);
  const uint32_t slot = j % S.NS;
  const uint32_t cnt = S.tl_cnt[slot * CNT_PAD];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x; b < cnt; b += stride) {
    const uint64_t i = b + threadIdx.x;
    bool want = false, first = false;
    uint32_t y = 0, v = INF32;
    if (i < cnt) {
      y = S.tl[(size_t)slot * S.n + i];
      v = S.pend[(size_t)slot * S.n + y];
      const uint32_t cur = S.ml[y];
      S.pend[(size_t)slot * S.n + y] = INF32;
      if (v < cur) {
        S.ml[y] = v;
        want = true;
        first = cur == INF32;
      }
    }
    touch(S, first, y);
    sweep_push_lanes(S, q, want, y, v, j);
  }
  slotq_flush(S, q);
}

// the pieces of long rows queued at distance j: one wave per piece; the label
// is the vertex's own (settled at j, unchanged until the next distance).  Also
// clears slot j (consumed) and the long-row counter of distance j + 1 (its
// last use, distance j - 1, is over).
__global__ __launch_bounds__(256) void k_sweep_heavy(SweepArgs S, uint32_t j) {
  SLOTQ_DECL(q);
  const int lane = lane_id();
  const uint32_t cnt = S.heavy_cnt[j & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S.tl_cnt[(j % S.NS) * CNT_PAD] = 0;
    S.heavy_cnt[(j + 1) & 1] = 0;
  }
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
  for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; i < cnt; i += nw) {
    uint64_t a0, a1;
    const uint32_t x = piece_arcs(S.heavy[i], S.row_ptr, &a0, &a1);
    const uint32_t lab = S.ml[x];
    const uint32_t R = S.Rg[seg_of(S.gid, x)];
    for (uint64_t b = a0; b < a1; b += 2 * WAVE) {
      const uint64_t i0 = b + lane, i1 = b + WAVE + lane;
      sweep_arcs2(S, q, j, i0 < a1, i0, lab, R, i1 < a1, i1, lab, R);
    }
  }
  slotq_flush(S, q);
}

__global__ void k_sweep_reset(SweepArgs S) {
  const uint32_t cnt = *S.touched_cnt;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * blockDim.x)
    S.ml[S.touched[i]] = INF32;
}

struct MisWork {
  SweepArgs S;
  const Graph *g;
  uint32_t *cbits;   // [n / 32] clients of the current step
  uint32_t *fbits;   // [n / 32] active facilities of the current round
  uint32_t *lab;     // [n] source labels
  uint32_t *act;     // [n] list of active facilities
  uint32_t *act2;    // [n]
  uint32_t *joined;  // [n]
  uint32_t *cov;     // [n]
  uint32_t *src;     // [n] sweep sources
  uint32_t *cnts;    // [8] device counters
};

enum class Toward { clients, facilities };

// blocks of a long-row sweep launch: twice the other frontier kernels'
// HEAVY_BLOCKS, 32 waves per CU on 256 CUs.  A hub piece keeps two groups of
// reads in flight per wave, and the extra waves add more: MIS 1.080 -> 0.954 s
// on the large weighted workload, timed on one box, identical results (four
// times gave the same)
constexpr uint32_t SWEEP_HEAVY_BLOCKS = 2 * HEAVY_BLOCKS;

// sweeps from at most this many sources skip the first readback of the
// frontier counts
constexpr uint32_t SWEEP_BLIND_SRC = 4096;

// run one sweep to completion; results in S.ml (caller resets afterwards).
// Toward::clients: from facilities f to every x with d(x, f) <= R (in-arcs);
// Toward::facilities: from clients c to every x with d(c, x) <= R (out-arcs).
// S.ml is exact at the vertices of the bitmap targets and at every vertex
// closer than R; a vertex at distance exactly R outside targets may keep no
// label.
static void sweep(Ctx &c, MisWork &M, const uint32_t *src, uint32_t nsrc, uint32_t R, Toward dir,
                  const uint32_t *targets) {
  SweepArgs &S = M.S;
  if (nsrc == 0) return;
  S.tbits = targets;
  const bool in = dir == Toward::clients;
  S.row_ptr = in ? M.g->in_ptr : M.g->row_ptr;
  S.col = in ? M.g->in_col : M.g->col;
  S.w = in ? M.g->in_w : M.g->w;
  k_sweep_init<<<(uint32_t)ceil_div((uint64_t)nsrc, 256), 256, 0, c.s>>>(S, src, nsrc, M.lab);
  FL_LAUNCH_CHECK();
  k_sweep_heavy<<<SWEEP_HEAVY_BLOCKS, 256, 0, c.s>>>(S, 0);
  FL_LAUNCH_CHECK();
  std::vector<uint32_t> h(S.NS);
  uint32_t j = 1;
  // few sources: run the first burst without reading the counts back (its
  // grid fits any frontier, and an empty distance costs one short launch)
  bool blind = nsrc <= SWEEP_BLIND_SRC;
  while (j <= R) {
    uint64_t pending = 1;
    uint32_t hmax = 0;
    if (!blind) {
      fetch_padded(c, h.data(), S.tl_cnt, S.NS);
      pending = 0;
      for (uint32_t s = 0; s < S.NS; ++s) {
        pending += h[s];
        hmax = std::max(hmax, h[s]);
      }
    }
    blind = false;
    if (!pending) break;
    // k_sweep_round reads its slot's count on the device, so 8 distances run
    // per host check (large frontiers too: MIS 1.093 -> 1.083 s on the large
    // weighted workload against a check after every distance of a frontier
    // above 65,536).  A frontier can grow from a handful of vertices to most
    // of the graph within a burst, so burst launches get a grid for any
    // frontier (the kernel strides over the count; blocks past it exit at
    // once).
    const uint32_t burst = 8u;
    const uint64_t want = std::max<uint64_t>(ceil_div((uint64_t)hmax * 2, 256),
                                             std::min<uint64_t>(ceil_div(S.n, 256), 2048));
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(want, 4), 8192);
    for (uint32_t b = 0; b < burst && j <= R; ++b, ++j) {
      k_sweep_round<<<blocks, 256, 0, c.s>>>(S, j);
      FL_LAUNCH_CHECK();
      k_sweep_heavy<<<SWEEP_HEAVY_BLOCKS, 256, 0, c.s>>>(S, j);
      FL_LAUNCH_CHECK();
    }
  }
  fill_u32(c, S.heavy_cnt, 2, 0);  // the last distance's long-row count
}

static void sweep_reset(Ctx &c, MisWork &M) {
  k_sweep_reset<<<1024, 256, 0, c.s>>>(M.S);
  FL_LAUNCH_CHECK();
  fill_u32(c, M.S.touched_cnt, 1, 0);
}

// ---- small per-round kernels -------------------------------------------------
// Priority of facility f: the fixed one (luby_round == 0), or for Luby's
// variant the one drawn for round r of the rung, a bijection keyed by
// SplitMix64(seed ^ (3 + 256 r)).
__device__ inline uint32_t priority_of(uint32_t f, const uint32_t *gid, const SegInfo *seg, uint32_t luby_round) {
  const SegInfo &sg = seg[seg_of(gid, f)];
  const PermKey key = luby_round ? perm_key(sg.seed, 3ull + 256ull * luby_round) : sg.pk;
  return perm_fwd(f - sg.base, key);
}
__global__ void k_set_key_labels(const uint32_t *list, uint32_t cnt, uint32_t *lab, const uint32_t *gid,
                                 const SegInfo *seg, uint32_t luby_round) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) lab[list[i]] = priority_of(list[i], gid, seg, luby_round);
}
__global__ void k_set_const_labels(const uint32_t *list, uint32_t cnt, uint32_t *lab, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) lab[list[i]] = v;
}
// clients of the rung: their pi_min (ml[c]) becomes their label; sources for
// sweep 2 are those with a value
__global__ void k_take_pmin(const uint32_t *cl, uint32_t ncl, const uint32_t *ml, uint32_t *lab,
                            uint32_t *src, uint32_t *nsrc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool want = false;
  uint32_t c = 0;
  if (i < ncl) {
    c = cl[i];
    const uint32_t v = ml[c];
    if (v != INF32) {
      lab[c] = v;
      want = true;
    }
  }
  const uint64_t m = __ballot(want);
  if (m) {
    const int lead = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane_id() == lead) base = atomicAdd(nsrc, (uint32_t)__popcll(m));
    base = __shfl(base, lead, WAVE);
    if (want) src[base + lanes_below(m)] = c;
  }
}
// join test: m(f) = ml[f]; join iff no client (INF) or m(f) == pi(f)
__global__ void k_join(const uint32_t *act, uint32_t na, const uint32_t *ml, const uint32_t *gid,
                       const SegInfo *seg, uint32_t luby_round, uint8_t *open, uint32_t *joined, uint32_t *nj,
                       uint32_t *rest, uint32_t *nr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool j = false, r = false;
  uint32_t f = 0;
  if (i < na) {
    f = act[i];
    const uint32_t m = ml[f];
    j = m == INF32 || m >= priority_of(f, gid, seg, luby_round);
    r = !j;
    if (j) open[f] = 1;
  }
  uint64_t mj = __ballot(j), mr = __ballot(r);
  uint32_t bj = 0, br = 0;
  if (lane_id() == 0) {
    if (mj) bj = atomicAdd(nj, (uint32_t)__popcll(mj));
    if (mr) br = atomicAdd(nr, (uint32_t)__popcll(mr));
  }
  bj = __shfl(bj, 0, WAVE);
  br = __shfl(br, 0, WAVE);
  if (j) joined[bj + lanes_below(mj)] = f;
  if (r) rest[br + lanes_below(mr)] = f;
}
// clients of the rung reached by a label (ml == 0) -> list
__global__ void k_collect_hit(const uint32_t *list, uint32_t cnt, const uint32_t *ml, uint32_t *out,
                              uint32_t *nout, int keep_hit) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool want = false;
  uint32_t x = 0;
  if (i < cnt) {
    x = list[i];
    const bool hit = ml[x] == 0;
    want = keep_hit ? hit : !hit;
  }
  const uint64_t m = __ballot(want);
  if (m) {
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(nout, (uint32_t)__popcll(m));
    base = __shfl(base, 0, WAVE);
    if (want) out[base + lanes_below(m)] = x;
  }
}

// per-(graph, rung) lists: counting sort by key koff[g] + t - 1 (t in 1..T[g])
__device__ inline bool rung_key(uint32_t v, const uint32_t *rung, const uint32_t *gid, const uint32_t *koff,
                                const uint32_t *Tg, uint32_t *key) {
  const uint32_t t = rung[v];
  const uint32_t g = seg_of(gid, v);
  if (t < 1 || t > Tg[g]) return false;
  *key = koff[g] + t - 1;
  return true;
}
// With few keys (K <= RK_LDS) a block counts in LDS first and adds one
// global atomic per key it saw: the per-rung counters are otherwise hit by
// every vertex of the rung.
constexpr uint32_t RK_LDS = 4096;
constexpr uint32_t RK_ITEMS = 16;  // vertices per thread in the LDS path
__global__ __launch_bounds__(256) void k_rung_count(uint32_t n, const uint32_t *rung, const uint32_t *gid,
                                                    const uint32_t *koff, const uint32_t *Tg, uint32_t K,
                                                    uint32_t *cnt) {
  __shared__ uint32_t lc[RK_LDS];
  uint32_t key;
  if (K > RK_LDS) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && rung_key((uint32_t)v, rung, gid, koff, Tg, &key)) atomicAdd(&cnt[key], 1u);
    return;
  }
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) lc[i] = 0;
  __syncthreads();
  const uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x * RK_ITEMS;
  for (uint32_t it = 0; it < RK_ITEMS; ++it) {
    const uint64_t v = v0 + (uint64_t)it * blockDim.x + threadIdx.x;
    if (v < n && rung_key((uint32_t)v, rung, gid, koff, Tg, &key)) atomicAdd(&lc[key], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x)
    if (lc[i]) atomicAdd(&cnt[i], lc[i]);
}
__global__ __launch_bounds__(256) void k_rung_scatter(uint32_t n, const uint32_t *rung, const uint32_t *gid,
                                                      const uint32_t *koff, const uint32_t *Tg, uint32_t K,
                                                      const uint64_t *off, uint32_t *cur, uint32_t *out) {
  __shared__ uint32_t lc[RK_LDS];
  uint32_t key;
  if (K > RK_LDS) {
    const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && rung_key((uint32_t)v, rung, gid, koff, Tg, &key))
      out[off[key] + atomicAdd(&cur[key], 1u)] = (uint32_t)v;
    return;
  }
  // local positions, then one reservation per key, then the writes
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) lc[i] = 0;
  __syncthreads();
  const uint64_t v0 = (uint64_t)blockIdx.x * blockDim.x * RK_ITEMS;
  uint32_t lpos[RK_ITEMS], keys[RK_ITEMS];
  for (uint32_t it = 0; it < RK_ITEMS; ++it) {
    const uint64_t v = v0 + (uint64_t)it * blockDim.x + threadIdx.x;
    keys[it] = INF32;
    if (v < n && rung_key((uint32_t)v, rung, gid, koff, Tg, &key)) {
      keys[it] = key;
      lpos[it] = atomicAdd(&lc[key], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < K; i += blockDim.x)
    if (lc[i]) lc[i] = atomicAdd(&cur[i], lc[i]);
  __syncthreads();
  for (uint32_t it = 0; it < RK_ITEMS; ++it) {
    const uint64_t v = v0 + (uint64_t)it * blockDim.x + threadIdx.x;
    if (keys[it] != INF32) out[off[keys[it]] + lc[keys[it]] + lpos[it]] = (uint32_t)v;
  }
}
// concatenate ranges [src + start, src + start + len) of a list; blockIdx.x
// picks the range, the blocks along y split it
__global__ void k_gather_ranges(const uint32_t *src, const uint64_t *rstart, const uint32_t *rlen,
                                const uint64_t *rdst, uint32_t *dst) {
  const uint32_t r = blockIdx.x;
  const uint64_t s0 = rstart[r], d0 = rdst[r];
  const uint32_t len = rlen[r];
  const uint64_t stride = (uint64_t)gridDim.y * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; i < len; i += stride) dst[d0 + i] = src[s0 + i];
}
// graphs whose facility of list[i] is active this round
__global__ void k_mark_graphs(const uint32_t *list, uint32_t cnt, const uint32_t *gid, uint32_t *flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) flag[seg_of(gid, list[i])] = 1u;
}
__global__ void k_guard_open(uint32_t n, const uint32_t *orung, uint8_t *open) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) open[v] = orung[v] == FL_RUNG_GUARD ? 1 : 0;
}
// bitmap membership of the vertices of a list (set or clear)
__global__ void k_mark_bits(const uint32_t *list, uint32_t cnt, uint32_t *bits, int set) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint32_t x = list[i];
  if (set) atomicOr(&bits[x >> 5], 1u << (x & 31));
  else atomicAnd(&bits[x >> 5], ~(1u << (x & 31)));
}
static void mark_bits(Ctx &c, const uint32_t *list, uint32_t cnt, uint32_t *bits, int set) {
  if (!cnt) return;
  k_mark_bits<<<(uint32_t)ceil_div(cnt, 256), 256, 0, c.s>>>(list, cnt, bits, set);
  FL_LAUNCH_CHECK();
}
__global__ void k_open_list(const uint32_t *list, uint32_t cnt, uint8_t *open) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) open[list[i]] = 1;
}

static void by_rung(Ctx &c, uint32_t n, const uint32_t *rung, const uint32_t *gid, const uint32_t *koff,
                    const uint32_t *Tg, uint32_t K, uint32_t *list, std::vector<uint64_t> &hoff) {
  uint32_t *cnt = c.arena->get<uint32_t>((size_t)K + 1);
  uint32_t *cur = c.arena->get<uint32_t>((size_t)K + 1);
  uint64_t *off = c.arena->get<uint64_t>((size_t)K + 2);
  fill_u32(c, cnt, K + 1, 0);
  fill_u32(c, cur, K + 1, 0);
  const uint32_t vb = (uint32_t)(K > RK_LDS ? ceil_div(n, 256) : ceil_div(n, 256 * RK_ITEMS));
  k_rung_count<<<vb, 256, 0, c.s>>>(n, rung, gid, koff, Tg, K, cnt);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, cnt, off, K);
  k_rung_scatter<<<vb, 256, 0, c.s>>>(n, rung, gid, koff, Tg, K, off, cur, list);
  FL_LAUNCH_CHECK();
  hoff.resize((size_t)K + 1);
  FL_HIP(hipMemcpyAsync(hoff.data(), off, hoff.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
}

static uint32_t read_u32(Ctx &c, const uint32_t *d) {
  FL_HIP(hipMemcpyAsync(c.h_status, d, 4, hipMemcpyDeviceToHost, c.s));
  c.sync();
  return (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
}

// Concatenates host-described ranges of `src` into `dst` on the device;
// returns the total length.
struct RangeBuf {
  uint64_t *start, *dst;
  uint32_t *len;
};
static uint32_t gather(Ctx &c, const uint32_t *src, const std::vector<std::pair<uint64_t, uint32_t>> &rs,
                       RangeBuf &rb, uint32_t *dst) {
  if (rs.empty()) return 0;
  const size_t R = rs.size();
  std::vector<uint64_t> hs(R), hd(R);
  std::vector<uint32_t> hl(R);
  uint64_t tot = 0;
  for (size_t i = 0; i < R; ++i) {
    hs[i] = rs[i].first;
    hl[i] = rs[i].second;
    hd[i] = tot;
    tot += rs[i].second;
  }
  FL_HIP(hipMemcpyAsync(rb.start, hs.data(), R * 8, hipMemcpyHostToDevice, c.s));
  FL_HIP(hipMemcpyAsync(rb.dst, hd.data(), R * 8, hipMemcpyHostToDevice, c.s));
  FL_HIP(hipMemcpyAsync(rb.len, hl.data(), R * 4, hipMemcpyHostToDevice, c.s));
  uint32_t maxlen = 1;
  for (size_t i = 0; i < R; ++i) maxlen = std::max(maxlen, hl[i]);
  const uint32_t cy = (uint32_t)std::min<uint64_t>(ceil_div(maxlen, 1024), 1024);
  k_gather_ranges<<<dim3((uint32_t)R, cy), 256, 0, c.s>>>(src, rb.start, rb.len, rb.dst, dst);
  FL_LAUNCH_CHECK();
  c.sync();  // the host vectors are released on return
  return (uint32_t)tot;
}

int mis_phase(Ctx &c, const MisIn &in, uint8_t *open, std::vector<uint32_t> &rounds_out) {
  const Graph &g = *in.g;
  const uint32_t n = g.n, G = in.G;
  const uint32_t NS = (g.w ? g.max_w : 1u) + 1;
  k_guard_open<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, in.orung, open);
  FL_LAUNCH_CHECK();
  rounds_out.assign(G, 0);
  // keys (graph, rung) -> koff[g] + t - 1
  std::vector<uint32_t> hkoff(G), hT(G);
  uint64_t K64 = 0;
  for (uint32_t q = 0; q < G; ++q) {
    hkoff[q] = (uint32_t)K64;
    hT[q] = in.rungs[q];
    K64 += in.rungs[q];
  }
  if (K64 == 0) return FL_OK;
  if (K64 >= 0xFFFFFFF0ull) return FL_ENOMEM;
  const uint32_t K = (uint32_t)K64;
  uint32_t *koff = c.arena->get<uint32_t>(G);
  uint32_t *Tg = c.arena->get<uint32_t>(G);
  FL_HIP(hipMemcpyAsync(koff, hkoff.data(), G * 4, hipMemcpyHostToDevice, c.s));
  FL_HIP(hipMemcpyAsync(Tg, hT.data(), G * 4, hipMemcpyHostToDevice, c.s));
  uint32_t *flist = c.arena->get<uint32_t>(n);
  uint32_t *clist = c.arena->get<uint32_t>(n);
  std::vector<uint64_t> foff, coff;
  by_rung(c, n, in.orung, in.gid, koff, Tg, K, flist, foff);
  by_rung(c, n, in.frz, in.gid, koff, Tg, K, clist, coff);

  MisWork M;
  M.S.n = n;
  M.S.NS = NS;
  M.S.gid = in.gid;
  uint32_t *d_R = c.arena->get<uint32_t>(G);
  M.S.Rg = d_R;
  M.g = &g;
  M.S.ml = c.arena->get<uint32_t>(n);
  M.S.pend = c.arena->get<uint32_t>((size_t)NS * n);
  M.S.tl = c.arena->get<uint32_t>((size_t)NS * n);
  M.S.tl_cnt = c.arena->get<uint32_t>((size_t)NS * CNT_PAD);
  M.S.touched = c.arena->get<uint32_t>(n);
  M.S.touched_cnt = c.arena->get<uint32_t>(1);
  M.S.heavy = c.arena->get<uint64_t>(piece_capacity(n, g.m));
  M.S.heavy_cnt = c.arena->get<uint32_t>(2);
  M.lab = c.arena->get<uint32_t>(n);
  M.act = c.arena->get<uint32_t>(n);
  M.act2 = c.arena->get<uint32_t>(n);
  M.joined = c.arena->get<uint32_t>(n);
  M.cov = c.arena->get<uint32_t>(n);
  M.src = c.arena->get<uint32_t>(n);
  M.cnts = c.arena->get<uint32_t>(8);
  const size_t nwords = ((size_t)n + 31) / 32;
  M.cbits = c.arena->get<uint32_t>(nwords);
  M.fbits = c.arena->get<uint32_t>(nwords);
  M.S.tbits = nullptr;
  uint32_t *ct_list = c.arena->get<uint32_t>(n);  // clients of the current step
  uint32_t *gact = c.arena->get<uint32_t>(G);     // graphs active in a round
  RangeBuf rb;
  rb.start = c.arena->get<uint64_t>(G);
  rb.dst = c.arena->get<uint64_t>(G);
  rb.len = c.arena->get<uint32_t>(G);
  fill_u32(c, M.S.ml, n, INF32);
  fill_u32(c, M.S.pend, (size_t)NS * n, INF32);
  fill_u32(c, M.S.tl_cnt, (size_t)NS * CNT_PAD, 0);
  fill_u32(c, M.S.touched_cnt, 1, 0);
  fill_u32(c, M.S.heavy_cnt, 2, 0);
  fill_u32(c, M.cbits, nwords, 0);
  fill_u32(c, M.fbits, nwords, 0);

  // each graph's non-empty rungs, in order
  std::vector<std::vector<uint32_t>> lists(G);
  size_t steps = 0;
  for (uint32_t q = 0; q < G; ++q) {
    for (uint32_t t = 1; t <= hT[q]; ++t) {
      const uint32_t key = hkoff[q] + t - 1;
      if (foff[key + 1] > foff[key]) lists[q].push_back(t);
    }
    steps = std::max(steps, lists[q].size());
  }
  const double one_eps = 1.0 + in.eps;
  std::vector<uint32_t> hR(G, 0), hact(G);
  std::vector<std::pair<uint64_t, uint32_t>> fr, cr, single;
  for (size_t i = 0; i < steps; ++i) {
    fr.clear();
    cr.clear();
    single.clear();
    uint32_t Rmax = 0;
    std::fill(hR.begin(), hR.end(), 0u);
    for (uint32_t q = 0; q < G; ++q) {
      if (i >= lists[q].size()) continue;
      const uint32_t t = lists[q][i];
      const uint32_t key = hkoff[q] + t - 1;
      const uint32_t nf = (uint32_t)(foff[key + 1] - foff[key]);
      if (nf == 1) {
        single.push_back({foff[key], 1u});
        rounds_out[q] += 1;
        continue;
      }
      fr.push_back({foff[key], nf});
      const uint32_t ncl = (uint32_t)(coff[key + 1] - coff[key]);
      if (ncl) cr.push_back({coff[key], ncl});
      const double rho = one_eps * (*in.lad)[q][t];
      // integer radius: d <= rho  <=>  d <= floor(rho)
      hR[q] = rho >= 4294967295.0 ? 0xFFFFFFFEu : (uint32_t)std::floor(rho);
      Rmax = std::max(Rmax, hR[q]);
    }
    if (!single.empty()) {
      const uint32_t ns1 = gather(c, flist, single, rb, M.act);
      k_open_list<<<(uint32_t)ceil_div(ns1, 256), 256, 0, c.s>>>(M.act, ns1, open);
      FL_LAUNCH_CHECK();
    }
    if (fr.empty()) continue;
    FL_HIP(hipMemcpyAsync(d_R, hR.data(), G * 4, hipMemcpyHostToDevice, c.s));
    uint32_t na = gather(c, flist, fr, rb, M.act);
    const uint32_t ncl = gather(c, clist, cr, rb, ct_list);
    const uint32_t *Ct = ct_list;
    mark_bits(c, Ct, ncl, M.cbits, 1);
    uint32_t guard_rounds = 0, step_round = 0;
    uint32_t nf_max = 0;
    for (auto &r : fr) nf_max = std::max(nf_max, r.second);
    while (na) {
      // the active facility of smallest priority of each graph joins every round
      if (++guard_rounds > nf_max + 1) return FL_EHIP;
      const uint32_t luby_round = in.luby ? ++step_round : 0u;
      if (G > 1) {
        fill_u32(c, gact, G, 0);
        k_mark_graphs<<<(uint32_t)ceil_div(na, 256), 256, 0, c.s>>>(M.act, na, in.gid, gact);
        FL_LAUNCH_CHECK();
        FL_HIP(hipMemcpyAsync(hact.data(), gact, G * 4, hipMemcpyDeviceToHost, c.s));
      }
      mark_bits(c, M.act, na, M.fbits, 1);
      // 1. pi_min at the clients of the rung
      k_set_key_labels<<<(uint32_t)ceil_div(na, 256), 256, 0, c.s>>>(M.act, na, M.lab, in.gid, in.seg,
                                                                     luby_round);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.act, na, Rmax, Toward::clients, M.cbits);
      if (G > 1) {
        for (uint32_t q = 0; q < G; ++q) rounds_out[q] += hact[q];
      } else {
        rounds_out[0] += 1;
      }
      fill_u32(c, M.cnts, 8, 0);
      if (ncl) {
        k_take_pmin<<<(uint32_t)ceil_div(ncl, 256), 256, 0, c.s>>>(Ct, ncl, M.S.ml, M.lab, M.src, M.cnts);
        FL_LAUNCH_CHECK();
      }
      sweep_reset(c, M);
      const uint32_t ns2 = read_u32(c, M.cnts);
      // 2. smallest pi_min around each active facility; joins
      sweep(c, M, M.src, ns2, Rmax, Toward::facilities, M.fbits);
      k_join<<<(uint32_t)ceil_div(na, 256), 256, 0, c.s>>>(M.act, na, M.S.ml, in.gid, in.seg, luby_round, open,
                                                           M.joined, M.cnts + 1, M.act2, M.cnts + 2);
      FL_LAUNCH_CHECK();
      sweep_reset(c, M);
      FL_HIP(hipMemcpyAsync(c.h_status, M.cnts, 16, hipMemcpyDeviceToHost, c.s));
      c.sync();
      const uint32_t nj = (uint32_t)(c.h_status[0] >> 32);
      const uint32_t nr = (uint32_t)(c.h_status[1] & 0xFFFFFFFFu);
      if (nr == 0) {
        mark_bits(c, M.act, na, M.fbits, 0);
        break;
      }
      // 3. clients covered by a joined facility
      k_set_const_labels<<<(uint32_t)ceil_div(nj, 256), 256, 0, c.s>>>(M.joined, nj, M.lab, 0);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.joined, nj, Rmax, Toward::clients, M.cbits);
      if (ncl) {
        k_collect_hit<<<(uint32_t)ceil_div(ncl, 256), 256, 0, c.s>>>(Ct, ncl, M.S.ml, M.cov, M.cnts + 3, 1);
        FL_LAUNCH_CHECK();
      }
      sweep_reset(c, M);
      const uint32_t ncov = read_u32(c, M.cnts + 3);
      // 4. facilities next to a covered client retire
      k_set_const_labels<<<(uint32_t)ceil_div(ncov ? ncov : 1, 256), 256, 0, c.s>>>(M.cov, ncov, M.lab, 0);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.cov, ncov, Rmax, Toward::facilities, M.fbits);  // read at the rest, a subset of act
      mark_bits(c, M.act, na, M.fbits, 0);  // before act is rewritten
      k_collect_hit<<<(uint32_t)ceil_div(nr, 256), 256, 0, c.s>>>(M.act2, nr, M.S.ml, M.act, M.cnts + 4, 0);
      FL_LAUNCH_CHECK();
      sweep_reset(c, M);
      na = read_u32(c, M.cnts + 4);
    }
    mark_bits(c, Ct, ncl, M.cbits, 0);
  }
  return FL_OK;
}

}  // namespace fl
