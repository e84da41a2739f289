// fl_open.hip -- the facility-opening loop (Alg. 4 with OpenFacilities,
// Alg. 5) on the GPU.
//
// Rung t uses alpha = a[t] (alpha grows before use).  For each unopened
// facility f the loop needs N(f, alpha): the HIP estimate of the unfrozen
// served clients within alpha of f, a predicated query over f's sketch
// (Sec. 4.5).  It is kept exactly as an integer in units of 2^-52 (split into
// two 64-bit words, fix52) over a "live list": the crossed sketch entries
// (distance <= alpha) whose client is still unfrozen, compacted in place at
// the front of f's sketch row.  Per rung:
//   light kernel  (thread per facility): when nothing crossed and no client
//                 froze in the previous rung, N is unchanged; update q and
//                 test the opening condition q >= c(f) directly.
//   heavy kernel  (16 lanes per facility): drop frozen clients from the live
//                 list when clients froze in the previous rung, append newly
//                 crossed entries, recompute N exactly, then update q with
//                 Eq. 2 (first rung, sequential sum in sketch order) or Eq. 3
//                 (eps * alpha * N) and test the opening condition.
//   distance to the open set: multi-source Bellman-Ford from the facilities
//                 opened in this rung.
//   freeze kernel (thread per vertex): unfrozen served clients within
//                 (1 + eps) alpha of an open facility freeze at this rung.
// Several graphs (a disjoint union) run the loop together: rung t is the same
// for every graph still running, alpha and the counters are per graph, and a
// graph leaves the loop when its own stopping rule holds.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fl_common.h"
#include "fl_open.h"

namespace fl {

// status counters per graph: field f of graph g, stripe s at
// [((g * OC_NFIELD + f) * stripes + s) * sstride]; a single graph stripes
// its counters over 64 words on separate 128-byte lines, so that the blocks'
// atomics do not queue on one line
enum { OC_HEAVY = 0, OC_OPENED, OC_FROZEN, OC_FINITE, OC_NUF_DEC, OC_LIVE, OC_NFIELD };

// per-graph parameters of the current rung
struct RungParam {
  double alpha, eps_alpha, ae, a0, a1, rho;
  uint32_t run;      // the graph evaluates this rung
  uint32_t frz_prev; // some client of the graph froze in the previous rung
  uint32_t freeze;   // the freeze kernel runs for the graph (it has open facilities)
  uint32_t stuck;    // the stall check runs for the graph
};

struct OpenArgs {
  uint32_t n, nF, cap;
  uint32_t stripes, sstride;
  const uint32_t *gid;        // graph of each vertex (nullptr: one graph)
  const SegInfo *seg;
  const RungParam *rp;        // [G]
  const uint32_t *fac_list;
  const uint32_t *fac_cost;   // vertex-indexed
  uint32_t *sk_rank;          // live region holds client ids
  uint32_t *sk_dist;
  uint32_t *thr;              // rows by facility index
  const uint32_t *cnt;
  const uint8_t *ceff;
  uint32_t *frz;              // vertex-indexed freeze rung
  uint32_t *orung;            // vertex-indexed open rung
  double *q;
  uint64_t *shi, *slo;
  uint32_t *cursor, *nlive, *nxt;
  double *nhat;
  uint8_t *state;
  uint32_t *heavy;            // [nF]
  uint32_t *heavy_cnt;        // [1]
  uint32_t *opened;           // [nF] vertex ids opened this rung
  uint32_t *opened_cnt;       // [1]
  uint32_t *ctr;              // [G * OC_NFIELD * stripes * sstride]
};

__device__ inline void ctr_add(const OpenArgs &A, uint32_t g, int field, uint32_t v) {
  if (v) atomicAdd(&A.ctr[(((size_t)g * OC_NFIELD + field) * A.stripes + (blockIdx.x % A.stripes)) * A.sstride], v);
}

// Block-aggregated counter adds of a single graph (every thread of a
// 256-thread block calls it, in uniform control flow): for fields f0, f1 and
// f2 (-1: none), the number of the block's threads with v0, v1 or v2 set, one
// atomic per block and field.
__device__ inline void block_ctr(const OpenArgs &A, int f0, bool v0, int f1, bool v1, int f2, bool v2) {
  __shared__ uint32_t s_c[3][256 / WAVE];
  const int wv = threadIdx.x / WAVE;
  const uint32_t c0 = (uint32_t)__popcll(__ballot(v0));
  const uint32_t c1 = (uint32_t)__popcll(__ballot(v1));
  const uint32_t c2 = (uint32_t)__popcll(__ballot(v2));
  if (lane_id() == 0) {
    s_c[0][wv] = c0;
    s_c[1][wv] = c1;
    s_c[2][wv] = c2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int i = (int)threadIdx.x;
    const int f = i == 0 ? f0 : (i == 1 ? f1 : f2);
    uint32_t tot = 0;
    for (int w = 0; w < 256 / WAVE; ++w) tot += s_c[i][w];
    if (f >= 0) ctr_add(A, 0, f, tot);
  }
  __syncthreads();  // s_c may be reused
}

// wave-aggregated append of x to list (lanes with want)
__device__ inline void wave_append(uint32_t *list, uint32_t *count, bool want, uint32_t x) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  const int lead = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == lead) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, lead, WAVE);
  if (want) list[base + lanes_below(m)] = x;
}

// Block-aggregated append (every thread of a 256-thread block calls it, in
// uniform control flow): one global atomic per block.  Used where most waves
// append, so that the waves do not queue on one counter.
__device__ inline void block_append(uint32_t *list, uint32_t *count, bool want, uint32_t x) {
  __shared__ uint32_t s_off[256 / WAVE];
  __shared__ uint32_t s_base;
  const int lane = lane_id();
  const int wv = threadIdx.x / WAVE;
  const uint64_t m = __ballot(want);
  if (lane == 0) s_off[wv] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int i = 0; i < 256 / WAVE; ++i) {
      const uint32_t cw = s_off[i];
      s_off[i] = tot;
      tot += cw;
    }
    s_base = tot ? atomicAdd(count, tot) : 0u;
  }
  __syncthreads();
  if (want) list[s_base + s_off[wv] + lanes_below(m)] = x;
  __syncthreads();  // s_off and s_base may be reused
}

__global__ void k_fac_init(OpenArgs A) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.nF) return;
  A.q[i] = 0.0;
  A.shi[i] = 0;
  A.slo[i] = 0;
  A.cursor[i] = 0;
  A.nlive[i] = 0;
  A.nxt[i] = 0;  // entry 0 of every sketch is the facility itself, at distance 0
  A.nhat[i] = 0.0;
  A.state[i] = 0;
}

// opening test and bookkeeping of a facility that opens at rung t
__device__ inline bool try_open(const OpenArgs &A, uint32_t fi, uint32_t f, double qn, uint32_t t) {
  if (qn >= (double)A.fac_cost[f]) {
    A.state[fi] = 1;
    A.orung[f] = t;
    return true;
  }
  return false;
}

// live lists up to this long are rescanned by the light kernel (a thread per
// facility); longer ones, and facilities with newly crossed entries, take
// the heavy kernel (16 lanes per facility)
constexpr uint32_t LIGHT_RESCAN = 32;

// 256 threads per block (block_append)
__global__ __launch_bounds__(256) void k_open_light(OpenArgs A, uint32_t t) {
  const uint32_t fi = blockIdx.x * blockDim.x + threadIdx.x;
  bool heavy = false, opened = false, nuf = false;
  uint32_t f = 0, g = 0;
  if (fi < A.nF && !A.state[fi]) {
    f = A.fac_list[fi];
    g = seg_of(A.gid, f);
    const RungParam &R = A.rp[g];
    if (R.run) {
      const uint32_t nx = A.nxt[fi];
      const uint32_t nl = A.nlive[fi];
      const bool rescan = R.frz_prev && nl > 0;
      heavy = (nx != INF32 && (double)nx <= R.alpha) || (rescan && nl > LIGHT_RESCAN);
      if (!heavy) {
        double nh = A.nhat[fi];
        if (rescan) {
          // a short live list: drop the clients that froze, as the heavy
          // kernel does (exact subtraction, entries after the first gap move)
          const size_t base = (size_t)f * A.cap, trow = (size_t)fi * A.cap;
          uint64_t rhi = 0, rlo = 0;
          uint32_t wpos = 0;
          for (uint32_t i = 0; i < nl; ++i) {
            const uint32_t id = A.sk_rank[base + i];
            if (A.frz[id] != FL_RUNG_NONE) {
              const Fix52 x = fix52_of(hip_weight(A.thr[trow + i]));
              rhi += x.hi;
              rlo += x.lo;
            } else {
              if (wpos != i) {
                A.sk_rank[base + wpos] = id;
                A.thr[trow + wpos] = A.thr[trow + i];
                A.sk_dist[base + wpos] = A.sk_dist[base + i];
              }
              ++wpos;
            }
          }
          if (wpos != nl) {
            const uint64_t shi = A.shi[fi] - rhi, slo = A.slo[fi] - rlo;
            A.shi[fi] = shi;
            A.slo[fi] = slo;
            A.nlive[fi] = wpos;
            nh = fix52_to_double(shi, slo);
            A.nhat[fi] = nh;
          }
        }
        // Eq. 3 with the current estimate (0 when nothing is live; at the
        // first rung nothing is live on this path, and an empty Eq. 2 sum is
        // 0 as well)
        const double inc = R.eps_alpha * nh;
        const double qn = A.q[fi] + inc;
        A.q[fi] = qn;
        opened = try_open(A, fi, f, qn, t);
        nuf = opened && A.ceff[f] && A.frz[f] == FL_RUNG_NONE;
      }
    }
  }
  // late rungs open facilities in most waves: block-level appends and counts
  block_append(A.heavy, A.heavy_cnt, heavy, fi);
  block_append(A.opened, A.opened_cnt, opened, f);
  if (A.gid) {
    if (opened) ctr_add(A, g, OC_OPENED, 1);
    if (nuf) ctr_add(A, g, OC_NUF_DEC, 1);
  } else {
    block_ctr(A, OC_OPENED, opened, OC_NUF_DEC, nuf, -1, false);
  }
}

// The heavy kernel gives each facility a group of OPEN_G lanes, so that a
// wave follows WAVE / OPEN_G facilities' chains of dependent loads (cursor,
// entries, the clients' freeze state, sums) at once.
constexpr int OPEN_G = 16;
static_assert(OPEN_G >= 2 && OPEN_G < 32 && (OPEN_G & (OPEN_G - 1)) == 0,
              "group masks are 32-bit: a power of two below 32 lanes");

// sum over the lane's OPEN_G-lane group (the group's lanes converged)
__device__ inline uint64_t group_sum_u64(uint64_t x) {
#pragma unroll
  for (int d = OPEN_G / 2; d >= 1; d >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)x, d, WAVE), hi = __shfl_xor((uint32_t)(x >> 32), d, WAVE);
    x += ((uint64_t)hi << 32) | lo;
  }
  return x;
}

__global__ __launch_bounds__(256) void k_open_heavy(OpenArgs A, uint32_t t) {
  const int lane = lane_id();
  const int sub = lane % OPEN_G;
  const int lead = lane - sub;  // the group's first lane
  const uint32_t below = (1u << sub) - 1u;
  // lanes of this group with cond set, as OPEN_G group-relative bits
  auto gballot = [&](bool cond) -> uint32_t {
    return (uint32_t)(__ballot(cond) >> lead) & ((1u << OPEN_G) - 1u);
  };
  const uint32_t nh = *A.heavy_cnt;
  constexpr uint32_t GPW = WAVE / OPEN_G;
  const uint64_t h0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE * GPW + (uint64_t)(lane / OPEN_G);
  const uint64_t ng = ((uint64_t)gridDim.x * blockDim.x) / WAVE * GPW;
  for (uint64_t h = h0; h < nh; h += ng) {
    const uint32_t fi = A.heavy[h];
    const uint32_t f = A.fac_list[fi];
    const uint32_t g = seg_of(A.gid, f);
    const RungParam &R = A.rp[g];
    const RankMap rm = rank_map(A.seg[g]);
    const double alpha = R.alpha;
    const int any_freeze_prev = R.frz_prev;
    const size_t base = (size_t)f * A.cap;
    const size_t trow = (size_t)fi * A.cap;
    const uint32_t c = A.cnt[f];
    uint32_t nl = A.nlive[fi];
    uint32_t cur = A.cursor[fi];
    uint64_t lhi = 0, llo = 0;  // weight added (crossed entries)
    uint64_t rhi = 0, rlo = 0;  // weight removed (clients that froze)
    const bool rescan = any_freeze_prev && nl > 0;
    if (rescan) {
      // drop the clients that froze: subtract their weights from the exact
      // sum and close the gaps (entries before the first gap stay in place)
      uint32_t wpos = 0;
      for (uint32_t b = 0; b < nl; b += OPEN_G) {
        const uint32_t i = b + sub;
        const bool valid = i < nl;
        const uint32_t id = valid ? A.sk_rank[base + i] : 0u;
        const bool gone = valid && A.frz[id] != FL_RUNG_NONE;
        const bool keep = valid && !gone;
        const uint32_t mk = gballot(keep);
        const uint32_t p = wpos + (uint32_t)__popc(mk & below);
        const bool move = keep && p != i;
        uint32_t T = 0, d = 0;
        if (gone || move) T = A.thr[trow + i];
        if (move) d = A.sk_dist[base + i];
        if (gone) {
          const Fix52 x = fix52_of(hip_weight(T));
          rhi += x.hi;
          rlo += x.lo;
        }
        if (move) {
          A.sk_rank[base + p] = id;
          A.thr[trow + p] = T;
          A.sk_dist[base + p] = d;
        }
        wpos += (uint32_t)__popc(mk);
      }
      nl = wpos;
    }
    // cross entries with distance <= alpha (entries are sorted by distance)
    while (cur < c) {
      const uint32_t j = cur + sub;
      const bool valid = j < c;
      uint32_t d = INF32;
      if (valid) d = A.sk_dist[base + j];
      const bool cross = valid && (double)d <= alpha;
      const uint32_t ncross = (uint32_t)__popc(gballot(cross));
      if (ncross == 0) break;
      bool keep = false;
      uint32_t id = 0, T = 0;
      if (cross) {
        id = id_of(A.sk_rank[base + j], rm);
        T = A.thr[trow + j];
        keep = A.ceff[id] && A.frz[id] == FL_RUNG_NONE;
      }
      const uint32_t mk = gballot(keep);
      if (keep) {
        const uint32_t p = nl + (uint32_t)__popc(mk & below);
        A.sk_rank[base + p] = id;
        A.thr[trow + p] = T;
        A.sk_dist[base + p] = d;
        const Fix52 x = fix52_of(hip_weight(T));
        lhi += x.hi;
        llo += x.lo;
      }
      nl += (uint32_t)__popc(mk);
      cur += ncross;
      if (ncross < (uint32_t)OPEN_G) break;
    }
    lhi = group_sum_u64(lhi);
    llo = group_sum_u64(llo);
    rhi = group_sum_u64(rhi);
    rlo = group_sum_u64(rlo);
    // each word is a sum over the live entries, so removing a subset keeps it
    // exact (no word goes below zero)
    uint64_t shi = A.shi[fi] - rhi + lhi;
    uint64_t slo = A.slo[fi] - rlo + llo;
    const double nh_ = fix52_to_double(shi, slo);
    if (sub == 0) {
      double inc;
      if (t == 1) {
        // Eq. 2: sum over the live entries, in sketch order, of
        // a_j ((1+eps) alpha - beta(d_j)); beta is a[0] or a[1] here
        double s = 0.0;
        for (uint32_t i = 0; i < nl; ++i) {
          const double dj = (double)A.sk_dist[base + i];
          const double b = dj <= R.a0 ? R.a0 : R.a1;
          s = s + hip_weight(A.thr[trow + i]) * (R.ae - b);
        }
        inc = s;
      } else {
        inc = R.eps_alpha * nh_;
      }
      A.shi[fi] = shi;
      A.slo[fi] = slo;
      A.nlive[fi] = nl;
      A.cursor[fi] = cur;
      A.nxt[fi] = cur < c ? A.sk_dist[base + cur] : INF32;
      A.nhat[fi] = nh_;
      const double qn = A.q[fi] + inc;
      A.q[fi] = qn;
      if (try_open(A, fi, f, qn, t)) {
        const uint32_t p = atomicAdd(A.opened_cnt, 1u);
        A.opened[p] = f;
        ctr_add(A, g, OC_OPENED, 1);
        if (A.ceff[f] && A.frz[f] == FL_RUNG_NONE) ctr_add(A, g, OC_NUF_DEC, 1);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Quiet rungs.  When no client froze in the previous rung, a rung in which no
// facility crosses its next sketch entry, none reaches its cost and no client
// comes within (1 + eps) alpha of the open set changes nothing but q:
// q += (eps alpha_t) N for every unopened facility, with N fixed.  The next
// rung with an event is found on the device and the quiet rungs before it
// are applied in one pass, in the same floating-point order as rung by rung.
// ---------------------------------------------------------------------------
constexpr uint32_t FF_WIN = 256;  // ladder rungs held on the device per look-ahead

struct FFArgs {
  const double *lw;     // [G * FF_WIN] a_g[t0 + i] of running graphs
  const uint8_t *run;   // [G] the graph is still in the loop
  uint32_t t0, nw;      // rungs t0 .. t0 + nw - 1
  double eps, one_eps;
  uint32_t *tev;        // earliest event rung (atomic min), t0 + nw if none
};

__global__ __launch_bounds__(256) void k_ff_scan_fac(OpenArgs A, FFArgs F) {
  const uint32_t fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= A.nF || A.state[fi]) return;
  const uint32_t f = A.fac_list[fi];
  const uint32_t g = seg_of(A.gid, f);
  if (!F.run[g]) return;
  const double *a = F.lw + (size_t)g * FF_WIN;
  uint32_t ev = F.nw;
  const uint32_t nx = A.nxt[fi];
  if (nx != INF32)
    for (uint32_t i = 0; i < F.nw; ++i)
      if ((double)nx <= a[i]) {
        ev = i;
        break;
      }
  double q = A.q[fi];
  const double nh = A.nhat[fi], c = (double)A.fac_cost[f];
  for (uint32_t i = 0; i < ev; ++i) {
    const double ea = F.eps * a[i];
    q = q + ea * nh;
    if (q >= c) {
      ev = i;
      break;
    }
  }
  if (ev < F.nw) atomicMin(F.tev, F.t0 + ev);
}

__global__ __launch_bounds__(256) void k_ff_scan_cli(OpenArgs A, FFArgs F, const uint64_t *dlab) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= A.n || !A.ceff[c] || A.frz[c] != FL_RUNG_NONE) return;
  const uint32_t g = seg_of(A.gid, (uint32_t)c);
  if (!F.run[g]) return;
  const uint64_t L = dlab[c];
  if (L == INF64) return;
  const double d = (double)(uint32_t)(L >> 32);
  const double *a = F.lw + (size_t)g * FF_WIN;
  for (uint32_t i = 0; i < F.nw; ++i)
    if (d <= F.one_eps * a[i]) {
      atomicMin(F.tev, F.t0 + i);
      return;
    }
}

// the quiet rungs t0 .. t0 + nr - 1
__global__ __launch_bounds__(256) void k_ff_apply(OpenArgs A, FFArgs F, uint32_t nr) {
  const uint32_t fi = blockIdx.x * blockDim.x + threadIdx.x;
  if (fi >= A.nF || A.state[fi]) return;
  const uint32_t g = seg_of(A.gid, A.fac_list[fi]);
  if (!F.run[g]) return;
  const double *a = F.lw + (size_t)g * FF_WIN;
  double q = A.q[fi];
  const double nh = A.nhat[fi];
  for (uint32_t i = 0; i < nr; ++i) {
    const double ea = F.eps * a[i];
    q = q + ea * nh;
  }
  A.q[fi] = q;
}

// opened facilities become sources at distance 0 (tie = own id)
__global__ void k_seed_opened(const uint32_t *opened, const uint32_t *cnt, uint64_t *lab) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < *cnt) {
    const uint32_t f = opened[i];
    lab[f] = (uint64_t)f;
  }
}

__global__ __launch_bounds__(256) void k_freeze(OpenArgs A, const uint64_t *dlab, uint32_t t,
                                                const uint32_t *fac_idx) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool froze = false, finite = false, nuf = false;
  uint32_t g = 0;
  if (c < A.n && A.ceff[c] && A.frz[c] == FL_RUNG_NONE && A.rp[g = seg_of(A.gid, (uint32_t)c)].freeze) {
    const uint64_t L = dlab[c];
    if (L != INF64) {
      const uint32_t d = (uint32_t)(L >> 32);
      if ((double)d <= A.rp[g].rho) {
        A.frz[c] = t;
        froze = true;
        const uint32_t fi = fac_idx[c];
        nuf = fi != INF32 && !A.state[fi];
      } else {
        finite = true;
      }
    }
  }
  if (A.gid) {
    const bool valid = c < A.n;
    if (valid) g = seg_of(A.gid, (uint32_t)c);
    seg_add32(A.ctr, valid, g, OC_FROZEN, OC_NFIELD, A.stripes, froze ? 1u : 0u);
    seg_add32(A.ctr, valid, g, OC_FINITE, OC_NFIELD, A.stripes, finite ? 1u : 0u);
    seg_add32(A.ctr, valid, g, OC_NUF_DEC, OC_NFIELD, A.stripes, nuf ? 1u : 0u);
  } else {
    block_ctr(A, OC_FROZEN, froze, OC_FINITE, finite, OC_NUF_DEC, nuf);
  }
}

// Does some unopened facility still have an unfrozen served client anywhere
// in its sketch?  (Stall check; run only when no unfrozen client can be
// reached by an open facility and no unopened facility is itself one.)
__global__ __launch_bounds__(256) void k_stuck_scan(OpenArgs A) {
  const int lane = lane_id();
  const uint64_t fi = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (fi >= A.nF || A.state[fi]) return;
  const uint32_t f = A.fac_list[fi];
  const uint32_t g = seg_of(A.gid, f);
  if (!A.rp[g].stuck) return;
  const RankMap rm = rank_map(A.seg[g]);
  const size_t base = (size_t)f * A.cap;
  const uint32_t nl = A.nlive[fi], cur = A.cursor[fi], c = A.cnt[f];
  bool live = false;
  for (uint32_t i = lane; i < nl; i += WAVE) live |= A.frz[A.sk_rank[base + i]] == FL_RUNG_NONE;
  for (uint32_t j = cur + lane; j < c; j += WAVE) {
    const uint32_t id = id_of(A.sk_rank[base + j], rm);
    live |= A.ceff[id] && A.frz[id] == FL_RUNG_NONE;
  }
  if (__ballot(live) && lane == 0) atomicAdd(&A.ctr[((size_t)g * OC_NFIELD + OC_LIVE) * A.stripes * A.sstride], 1u);
}

// graphs flagged in gflag[g] & 1: stall guard; & 2: end phase
__global__ void k_guard(uint32_t n, const uint32_t *gid, const uint8_t *gflag, const uint8_t *ceff, uint32_t *frz,
                        uint32_t *orung, const uint64_t *gam) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !(gflag[seg_of(gid, (uint32_t)c)] & 1) || !ceff[c] || frz[c] != FL_RUNG_NONE) return;
  const uint32_t f = (uint32_t)(gam[c] & 0xFFFFFFFFu);
  orung[f] = FL_RUNG_GUARD;
  frz[c] = FL_RUNG_GUARD;
}

__global__ void k_endphase(uint32_t n, const uint32_t *gid, const uint8_t *gflag, const uint8_t *ceff,
                           uint32_t *frz) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && (gflag[seg_of(gid, (uint32_t)c)] & 2) && ceff[c] && frz[c] == FL_RUNG_NONE) frz[c] = FL_RUNG_END;
}

// per-graph sums of the striped counters
static void read_ctr(Ctx &c, const OpenArgs &A, uint32_t G, std::vector<uint64_t> &out) {
  std::vector<uint32_t> h((size_t)G * OC_NFIELD * A.stripes * A.sstride);
  FL_HIP(hipMemcpyAsync(h.data(), A.ctr, h.size() * 4, hipMemcpyDeviceToHost, c.s));
  c.sync();
  out.assign((size_t)G * OC_NFIELD, 0);
  for (size_t i = 0; i < out.size(); ++i)
    for (uint32_t s = 0; s < A.stripes; ++s) out[i] += h[(i * A.stripes + s) * A.sstride];
}

int open_phase(Ctx &c, const OpenIn &in, OpenOut &out) {
  const Graph &g = *in.g;
  const uint32_t n = g.n, nF = in.nF, G = in.G;
  OpenArgs A{};
  A.n = n;
  A.nF = nF;
  A.cap = in.ads->cap;
  // one graph: 64 stripes, 32 words (128 B) apart; a union: one plain
  // counter per graph and field (seg_add32 indexes it unstrided)
  A.stripes = G == 1 ? 64 : 1;
  A.sstride = G == 1 ? 32 : 1;
  A.gid = in.gid;
  A.seg = in.seg;
  A.fac_list = in.fac_list;
  A.fac_cost = in.fac_cost;
  A.sk_rank = in.ads->sk_rank;
  A.sk_dist = in.ads->sk_dist;
  A.thr = in.ads->thr;
  A.cnt = in.ads->cnt;
  A.ceff = in.ceff;
  A.frz = out.frz;
  A.orung = out.orung;
  A.q = out.q;
  A.shi = c.arena->get<uint64_t>(nF);
  A.slo = c.arena->get<uint64_t>(nF);
  A.cursor = c.arena->get<uint32_t>(nF);
  A.nlive = c.arena->get<uint32_t>(nF);
  A.nxt = c.arena->get<uint32_t>(nF);
  A.nhat = c.arena->get<double>(nF);
  A.state = c.arena->get<uint8_t>(nF);
  A.heavy = c.arena->get<uint32_t>(nF);
  A.opened = c.arena->get<uint32_t>(nF);
  uint32_t *cnts = c.arena->get<uint32_t>(2);
  A.heavy_cnt = cnts;
  A.opened_cnt = cnts + 1;
  const size_t ctr_words = (size_t)G * OC_NFIELD * A.stripes * A.sstride;
  A.ctr = c.arena->get<uint32_t>(ctr_words);
  RungParam *d_rp = c.arena->get<RungParam>(G);
  A.rp = d_rp;
  uint8_t *d_gflag = c.arena->get<uint8_t>(G);
  double *d_lw = c.arena->get<double>((size_t)G * FF_WIN);
  uint8_t *d_run = c.arena->get<uint8_t>(G);
  uint32_t *d_tev = c.arena->get<uint32_t>(1);
  std::vector<double> h_lw((size_t)G * FF_WIN);
  std::vector<uint8_t> h_run(G);
  uint64_t *dlab = c.arena->get<uint64_t>(n);
  fill_u64(c, dlab, n, INF64);
  fill_u32(c, out.frz, n, FL_RUNG_NONE);
  fill_u32(c, out.orung, n, FL_RUNG_NONE);
  if (nF) {
    k_fac_init<<<(uint32_t)ceil_div(nF, 256), 256, 0, c.s>>>(A);
    FL_LAUNCH_CHECK();
  }
  SsspWork wk;
  sssp_alloc(c, wk, n, g.m);

  const double one_eps = 1.0 + in.eps;
  // host state per graph
  std::vector<uint64_t> nO(G, 0), nU(in.nCeff), nUF(in.nUF0), finite_unfrozen(G, 0);
  std::vector<uint8_t> frz_prev(G, 0), done(G, 0), gflag(G, 0);
  std::vector<RungParam> rp(G);
  out.rungs.assign(G, 0);
  out.rc.assign(G, FL_OK);
  for (uint32_t q = 0; q < G; ++q) done[q] = !(nO[q] < in.nF_g[q] && nU[q] > 0);
  uint32_t t = 0;
  const uint32_t fblocks = (uint32_t)ceil_div(nF ? nF : 1, 256);
  const uint32_t hblocks = (uint32_t)std::min<uint64_t>(ceil_div((uint64_t)(nF ? nF : 1) * WAVE, 256), 4096);
  const uint32_t vblocks = (uint32_t)ceil_div(n, 256);
  std::vector<uint64_t> ctr;
  auto upload = [&]() {
    FL_HIP(hipMemcpyAsync(d_rp, rp.data(), G * sizeof(RungParam), hipMemcpyHostToDevice, c.s));
  };
  for (;;) {
    // stall check for the running graphs with nothing in reach
    bool any_stuck = false;
    for (uint32_t q = 0; q < G; ++q) {
      rp[q] = RungParam{};
      rp[q].stuck = !done[q] && finite_unfrozen[q] == 0 && nUF[q] == 0;
      any_stuck |= rp[q].stuck != 0;
    }
    if (any_stuck) {
      upload();
      fill_u32(c, A.ctr, ctr_words, 0);
      k_stuck_scan<<<(uint32_t)ceil_div((uint64_t)(nF ? nF : 1) * WAVE, 256), 256, 0, c.s>>>(A);
      FL_LAUNCH_CHECK();
      read_ctr(c, A, G, ctr);
      for (uint32_t q = 0; q < G; ++q)
        if (rp[q].stuck && ctr[(size_t)q * OC_NFIELD + OC_LIVE] == 0) {
          gflag[q] |= 1;  // stall guard
          nU[q] = 0;
          done[q] = 1;
        }
    }
    bool any = false;
    for (uint32_t q = 0; q < G; ++q) any |= !done[q];
    if (!any) break;
    // skip the quiet rungs before the next event (not the first rung, which
    // uses Eq. 2, and not right after a freeze, which changes N)
    bool can_ff = t >= 1 && nF > 0;
    bool any_open = false;
    for (uint32_t q = 0; q < G && can_ff; ++q) {
      if (done[q]) continue;
      can_ff = !frz_prev[q];
      any_open |= nO[q] > 0;
    }
    if (can_ff) {
      const uint32_t t0 = t + 1;
      for (uint32_t q = 0; q < G && can_ff; ++q) {
        h_run[q] = !done[q];
        std::vector<double> &lad = (*in.lad)[q];
        if (!h_run[q]) continue;
        while (lad.size() < (size_t)t0 + FF_WIN) lad.push_back(lad.back() * one_eps);
        for (uint32_t i = 0; i < FF_WIN; ++i) {
          const double a = lad[t0 + i];
          if (!std::isfinite(a)) can_ff = false;  // the rung loop reports the overflow
          h_lw[(size_t)q * FF_WIN + i] = a;
        }
      }
      if (can_ff) {
        FL_HIP(hipMemcpyAsync(d_lw, h_lw.data(), h_lw.size() * 8, hipMemcpyHostToDevice, c.s));
        FL_HIP(hipMemcpyAsync(d_run, h_run.data(), G, hipMemcpyHostToDevice, c.s));
        fill_u32(c, d_tev, 1, t0 + FF_WIN);
        FFArgs F{d_lw, d_run, t0, FF_WIN, in.eps, one_eps, d_tev};
        k_ff_scan_fac<<<fblocks, 256, 0, c.s>>>(A, F);
        FL_LAUNCH_CHECK();
        if (any_open) {
          k_ff_scan_cli<<<vblocks, 256, 0, c.s>>>(A, F, dlab);
          FL_LAUNCH_CHECK();
        }
        FL_HIP(hipMemcpyAsync(c.h_status, d_tev, 4, hipMemcpyDeviceToHost, c.s));
        c.sync();
        const uint32_t tev = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
        if (tev > t0) {
          k_ff_apply<<<fblocks, 256, 0, c.s>>>(A, F, tev - t0);
          FL_LAUNCH_CHECK();
          t = tev - 1;
          for (uint32_t q = 0; q < G; ++q)
            if (!done[q]) out.rungs[q] = t;
        }
      }
    }
    ++t;
    for (uint32_t q = 0; q < G; ++q) {
      RungParam &R = rp[q];
      R = RungParam{};
      if (done[q]) continue;
      std::vector<double> &lad = (*in.lad)[q];
      while (lad.size() <= t) lad.push_back(lad.back() * one_eps);
      const double alpha = lad[t];
      if (!std::isfinite(alpha)) {
        out.rc[q] = FL_ERANGE;
        done[q] = 1;
        continue;
      }
      R.alpha = alpha;
      R.eps_alpha = in.eps * alpha;
      R.ae = one_eps * alpha;
      R.a0 = lad[0];
      R.a1 = lad[1];
      R.rho = one_eps * alpha;
      R.run = 1;
      R.frz_prev = frz_prev[q];
      out.rungs[q] = t;
    }
    upload();
    fill_u32(c, cnts, 2, 0);
    fill_u32(c, A.ctr, ctr_words, 0);
    k_open_light<<<fblocks, 256, 0, c.s>>>(A, t);
    FL_LAUNCH_CHECK();
    k_open_heavy<<<hblocks, 256, 0, c.s>>>(A, t);
    FL_LAUNCH_CHECK();
    read_ctr(c, A, G, ctr);
    uint64_t opened = 0;
    bool any_freeze = false;
    for (uint32_t q = 0; q < G; ++q) {
      if (!rp[q].run) continue;
      const uint64_t o = ctr[(size_t)q * OC_NFIELD + OC_OPENED];
      opened += o;
      nO[q] += o;
      nUF[q] -= ctr[(size_t)q * OC_NFIELD + OC_NUF_DEC];
      frz_prev[q] = 0;
      rp[q].freeze = nO[q] > 0;
      any_freeze |= rp[q].freeze != 0;
    }
    if (opened) {
      k_seed_opened<<<(uint32_t)ceil_div(opened, 256), 256, 0, c.s>>>(A.opened, A.opened_cnt, dlab);
      FL_LAUNCH_CHECK();
      sssp_run(c, g, dlab, A.opened, (uint32_t)opened, wk, 0);
    }
    if (any_freeze) {
      upload();
      fill_u32(c, A.ctr, ctr_words, 0);
      k_freeze<<<vblocks, 256, 0, c.s>>>(A, dlab, t, in.fac_idx);
      FL_LAUNCH_CHECK();
      read_ctr(c, A, G, ctr);
      for (uint32_t q = 0; q < G; ++q) {
        if (!rp[q].freeze) continue;
        const uint64_t *cq = &ctr[(size_t)q * OC_NFIELD];
        nU[q] -= cq[OC_FROZEN];
        nUF[q] -= cq[OC_NUF_DEC];
        finite_unfrozen[q] = cq[OC_FINITE];
        frz_prev[q] = cq[OC_FROZEN] > 0;
      }
    }
    for (uint32_t q = 0; q < G; ++q)
      if (rp[q].run && !(nO[q] < in.nF_g[q] && nU[q] > 0)) done[q] = 1;
  }
  out.nO = nO;
  bool any_flag = false;
  for (uint32_t q = 0; q < G; ++q) {
    if (nO[q] == in.nF_g[q] && nU[q] > 0 && out.rc[q] == FL_OK) gflag[q] |= 2;  // end phase
    any_flag |= gflag[q] != 0;
  }
  if (any_flag) {
    FL_HIP(hipMemcpyAsync(d_gflag, gflag.data(), G, hipMemcpyHostToDevice, c.s));
    k_guard<<<vblocks, 256, 0, c.s>>>(n, in.gid, d_gflag, in.ceff, out.frz, out.orung, in.gam_lab);
    FL_LAUNCH_CHECK();
    k_endphase<<<vblocks, 256, 0, c.s>>>(n, in.gid, d_gflag, in.ceff, out.frz);
    FL_LAUNCH_CHECK();
    c.sync();  // gflag is read by the copy above
  }
  // q by vertex for the caller's diagnostics is scattered later
  return FL_OK;
}

}  // namespace fl
