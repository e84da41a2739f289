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
// priority order.  A sweep computes, for every vertex x, the minimum label
// over sources within distance R of x.  It runs in distance order (round j
// settles labels at distance exactly j) with one pending-label array per
// distance slot modulo max_w + 1, so a label is forwarded only when it
// lowers a vertex's current minimum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fl_common.h"
#include "fl_mis.h"

namespace fl {

struct SweepArgs {
  uint32_t n, NS;
  const uint64_t *row_ptr;
  const uint32_t *col;
  const uint32_t *w;
  uint32_t *ml;       // [n] current minimum label (INF32 = none)
  uint32_t *pend;     // [NS * n] pending label per slot
  uint32_t *tl;       // [NS * n] vertices with a pending label per slot
  uint32_t *tl_cnt;   // [NS]
  uint32_t *touched;  // [n] vertices whose ml was set
  uint32_t *touched_cnt;
};

// push label lab from x (settled at distance j) to its neighbours
__device__ inline void sweep_push(const SweepArgs &S, uint32_t x, uint32_t lab, uint32_t j, uint32_t R) {
  const int lane = lane_id();
  const uint64_t a0 = S.row_ptr[x], a1 = S.row_ptr[x + 1];
  for (uint64_t b = a0; b < a1; b += WAVE) {
    const uint64_t a = b + lane;
    bool add = false;
    uint32_t y = 0, s = 0;
    if (a < a1) {
      y = S.col[a];
      const uint32_t wv = S.w ? S.w[a] : 1u;
      if ((uint64_t)j + wv <= R) {
        s = (j + wv) % S.NS;
        uint32_t *p = &S.pend[(size_t)s * S.n + y];
        if (lab < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          const uint32_t old = atomicMin(p, lab);
          add = old == INF32;
        }
      }
    }
    // append y to tl[s] (group lanes by slot)
    uint64_t pendm = __ballot(add);
    while (pendm) {
      const int lead = __ffsll((long long)pendm) - 1;
      const uint32_t sl = __shfl(s, lead, WAVE);
      const bool mine = add && s == sl;
      const uint64_t grp = __ballot(mine);
      uint32_t base = 0;
      if (lane == lead) base = atomicAdd(&S.tl_cnt[sl], (uint32_t)__popcll(grp));
      base = __shfl(base, lead, WAVE);
      if (mine) {
        S.tl[(size_t)sl * S.n + base + lanes_below(grp)] = y;
        add = false;
      }
      pendm &= ~grp;
    }
  }
}

// sources: set ml and push at distance 0 (one wave per source)
__global__ __launch_bounds__(256) void k_sweep_init(SweepArgs S, const uint32_t *src, uint32_t nsrc,
                                                    const uint32_t *lab, uint32_t R) {
  const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (i >= nsrc) return;
  const uint32_t x = src[i];
  const uint32_t l = lab[x];
  if (lane_id() == 0 && l != INF32) {
    S.ml[x] = l;
    const uint32_t p = atomicAdd(S.touched_cnt, 1u);
    S.touched[p] = x;
  }
  sweep_push(S, x, l, 0, R);
}

__global__ __launch_bounds__(256) void k_sweep_round(SweepArgs S, uint32_t j, uint32_t R) {
  const uint32_t slot = j % S.NS;
  const uint32_t cnt = S.tl_cnt[slot];
  const uint64_t wid = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
  for (uint64_t i = wid; i < cnt; i += nw) {
    const uint32_t y = S.tl[(size_t)slot * S.n + i];
    const uint32_t v = S.pend[(size_t)slot * S.n + y];
    const uint32_t cur = S.ml[y];
    if (lane_id() == 0) S.pend[(size_t)slot * S.n + y] = INF32;
    if (v < cur) {
      if (lane_id() == 0) {
        S.ml[y] = v;
        if (cur == INF32) {
          const uint32_t p = atomicAdd(S.touched_cnt, 1u);
          S.touched[p] = y;
        }
      }
      sweep_push(S, y, v, j, R);
    }
  }
}

__global__ void k_sweep_reset(SweepArgs S) {
  const uint32_t cnt = *S.touched_cnt;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (uint64_t)gridDim.x * blockDim.x)
    S.ml[S.touched[i]] = INF32;
}

struct MisWork {
  SweepArgs S;
  uint32_t *lab;     // [n] source labels
  uint32_t *pm;      // [n] pi_min of clients
  uint32_t *act;     // [n] list of active facilities
  uint32_t *act2;    // [n]
  uint32_t *joined;  // [n]
  uint32_t *cov;     // [n]
  uint32_t *src;     // [n] sweep sources
  uint32_t *cnts;    // [8] device counters
};

// run one sweep to completion; results in S.ml (caller resets afterwards)
static void sweep(Ctx &c, MisWork &M, const uint32_t *src, uint32_t nsrc, uint32_t R) {
  SweepArgs &S = M.S;
  if (nsrc == 0) return;
  k_sweep_init<<<(uint32_t)ceil_div((uint64_t)nsrc * WAVE, 256), 256, 0, c.s>>>(S, src, nsrc, M.lab, R);
  FL_LAUNCH_CHECK();
  std::vector<uint32_t> h(S.NS);
  for (uint32_t j = 1; j <= R; ++j) {
    FL_HIP(hipMemcpyAsync(h.data(), S.tl_cnt, S.NS * 4, hipMemcpyDeviceToHost, c.s));
    c.sync();
    uint64_t pending = 0;
    for (uint32_t s = 0; s < S.NS; ++s) pending += h[s];
    if (!pending) break;
    const uint32_t slot = j % S.NS;
    const uint32_t cnt = h[slot];
    if (cnt) {
      const uint32_t blocks = (uint32_t)std::min<uint64_t>(ceil_div((uint64_t)cnt * WAVE, 256), 8192);
      k_sweep_round<<<blocks, 256, 0, c.s>>>(S, j, R);
      FL_LAUNCH_CHECK();
      fill_u32(c, S.tl_cnt + slot, 1, 0);
    }
  }
}

static void sweep_reset(Ctx &c, MisWork &M) {
  k_sweep_reset<<<1024, 256, 0, c.s>>>(M.S);
  FL_LAUNCH_CHECK();
  fill_u32(c, M.S.touched_cnt, 1, 0);
}

// ---- small per-round kernels -------------------------------------------------
__global__ void k_set_key_labels(const uint32_t *list, uint32_t cnt, uint32_t *lab, PermKey pk) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) lab[list[i]] = perm_fwd(list[i], pk);
}
__global__ void k_set_const_labels(const uint32_t *list, uint32_t cnt, uint32_t *lab, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) lab[list[i]] = v;
}
// clients of the rung: pm[c] = ml[c]; sources for sweep 2 are those with a value
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
__global__ void k_join(const uint32_t *act, uint32_t na, const uint32_t *ml, PermKey pk, uint8_t *open,
                       uint32_t *joined, uint32_t *nj, uint32_t *rest, uint32_t *nr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool j = false, r = false;
  uint32_t f = 0;
  if (i < na) {
    f = act[i];
    const uint32_t m = ml[f];
    j = m == INF32 || m >= perm_fwd(f, pk);
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

// per-rung lists: counting sort by rung value
__global__ void k_rung_count(uint32_t n, const uint32_t *rung, uint32_t T, uint32_t *cnt) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const uint32_t t = rung[v];
    if (t >= 1 && t <= T) atomicAdd(&cnt[t], 1u);
  }
}
__global__ void k_rung_scatter(uint32_t n, const uint32_t *rung, uint32_t T, const uint64_t *off,
                               uint32_t *cur, uint32_t *out) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const uint32_t t = rung[v];
    if (t >= 1 && t <= T) out[off[t] + atomicAdd(&cur[t], 1u)] = (uint32_t)v;
  }
}
__global__ void k_guard_open(uint32_t n, const uint32_t *orung, uint8_t *open) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) open[v] = orung[v] == FL_RUNG_GUARD ? 1 : 0;
}
__global__ void k_open_one(const uint32_t *list, uint8_t *open) { open[list[0]] = 1; }

static void by_rung(Ctx &c, uint32_t n, const uint32_t *rung, uint32_t T, uint32_t *list,
                    std::vector<uint64_t> &hoff) {
  uint32_t *cnt = c.arena->get<uint32_t>((size_t)T + 2);
  uint32_t *cur = c.arena->get<uint32_t>((size_t)T + 2);
  uint64_t *off = c.arena->get<uint64_t>((size_t)T + 3);
  fill_u32(c, cnt, T + 2, 0);
  fill_u32(c, cur, T + 2, 0);
  const uint32_t vb = (uint32_t)ceil_div(n, 256);
  k_rung_count<<<vb, 256, 0, c.s>>>(n, rung, T, cnt);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, cnt, off, T + 2);
  k_rung_scatter<<<vb, 256, 0, c.s>>>(n, rung, T, off, cur, list);
  FL_LAUNCH_CHECK();
  hoff.resize((size_t)T + 3);
  FL_HIP(hipMemcpyAsync(hoff.data(), off, hoff.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
}

static uint32_t read_u32(Ctx &c, const uint32_t *d) {
  FL_HIP(hipMemcpyAsync(c.h_status, d, 4, hipMemcpyDeviceToHost, c.s));
  c.sync();
  return (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
}

int mis_phase(Ctx &c, const MisIn &in, uint8_t *open, uint32_t *rounds_out) {
  const Graph &g = *in.g;
  const uint32_t n = g.n, T = in.rungs;
  const uint32_t NS = (g.w ? g.max_w : 1u) + 1;
  k_guard_open<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, in.orung, open);
  FL_LAUNCH_CHECK();
  *rounds_out = 0;
  if (T == 0) return FL_OK;
  uint32_t *flist = c.arena->get<uint32_t>(n);
  uint32_t *clist = c.arena->get<uint32_t>(n);
  std::vector<uint64_t> foff, coff;
  by_rung(c, n, in.orung, T, flist, foff);
  by_rung(c, n, in.frz, T, clist, coff);

  MisWork M;
  M.S.n = n;
  M.S.NS = NS;
  M.S.row_ptr = g.row_ptr;
  M.S.col = g.col;
  M.S.w = g.w;
  M.S.ml = c.arena->get<uint32_t>(n);
  M.S.pend = c.arena->get<uint32_t>((size_t)NS * n);
  M.S.tl = c.arena->get<uint32_t>((size_t)NS * n);
  M.S.tl_cnt = c.arena->get<uint32_t>(NS);
  M.S.touched = c.arena->get<uint32_t>(n);
  M.S.touched_cnt = c.arena->get<uint32_t>(1);
  M.lab = c.arena->get<uint32_t>(n);
  M.pm = c.arena->get<uint32_t>(n);
  M.act = c.arena->get<uint32_t>(n);
  M.act2 = c.arena->get<uint32_t>(n);
  M.joined = c.arena->get<uint32_t>(n);
  M.cov = c.arena->get<uint32_t>(n);
  M.src = c.arena->get<uint32_t>(n);
  M.cnts = c.arena->get<uint32_t>(8);
  fill_u32(c, M.S.ml, n, INF32);
  fill_u32(c, M.S.pend, (size_t)NS * n, INF32);
  fill_u32(c, M.S.tl_cnt, NS, 0);
  fill_u32(c, M.S.touched_cnt, 1, 0);

  const double one_eps = 1.0 + in.eps;
  uint32_t total_rounds = 0;
  for (uint32_t t = 1; t <= T; ++t) {
    const uint32_t nf = (uint32_t)(foff[t + 1] - foff[t]);
    if (nf == 0) continue;
    const uint32_t *Ft = flist + foff[t];
    if (nf == 1) {
      k_open_one<<<1, 1, 0, c.s>>>(Ft, open);
      FL_LAUNCH_CHECK();
      total_rounds += 1;
      continue;
    }
    const uint32_t ncl = (uint32_t)(coff[t + 1] - coff[t]);
    const uint32_t *Ct = clist + coff[t];
    const double rho = one_eps * (*in.lad)[t];
    // integer radius: d <= rho  <=>  d <= floor(rho)
    const uint32_t R = rho >= 4294967295.0 ? 0xFFFFFFFEu : (uint32_t)std::floor(rho);
    FL_HIP(hipMemcpyAsync(M.act, Ft, (size_t)nf * 4, hipMemcpyDeviceToDevice, c.s));
    uint32_t na = nf;
    uint32_t guard_rounds = 0;
    while (na) {
      // the active facility of smallest priority joins every round
      if (++guard_rounds > nf + 1) return FL_EHIP;
      ++total_rounds;
      // 1. pi_min at the clients of the rung
      k_set_key_labels<<<(uint32_t)ceil_div(na, 256), 256, 0, c.s>>>(M.act, na, M.lab, in.pk);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.act, na, R);
      fill_u32(c, M.cnts, 8, 0);
      if (ncl) {
        k_take_pmin<<<(uint32_t)ceil_div(ncl, 256), 256, 0, c.s>>>(Ct, ncl, M.S.ml, M.lab, M.src, M.cnts);
        FL_LAUNCH_CHECK();
      }
      sweep_reset(c, M);
      const uint32_t ns2 = read_u32(c, M.cnts);
      // 2. smallest pi_min around each active facility; joins
      sweep(c, M, M.src, ns2, R);
      k_join<<<(uint32_t)ceil_div(na, 256), 256, 0, c.s>>>(M.act, na, M.S.ml, in.pk, open, M.joined,
                                                           M.cnts + 1, M.act2, M.cnts + 2);
      FL_LAUNCH_CHECK();
      sweep_reset(c, M);
      FL_HIP(hipMemcpyAsync(c.h_status, M.cnts, 16, hipMemcpyDeviceToHost, c.s));
      c.sync();
      const uint32_t nj = (uint32_t)(c.h_status[0] >> 32);
      const uint32_t nr = (uint32_t)(c.h_status[1] & 0xFFFFFFFFu);
      if (nr == 0) break;
      // 3. clients covered by a joined facility
      k_set_const_labels<<<(uint32_t)ceil_div(nj, 256), 256, 0, c.s>>>(M.joined, nj, M.lab, 0);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.joined, nj, R);
      if (ncl) {
        k_collect_hit<<<(uint32_t)ceil_div(ncl, 256), 256, 0, c.s>>>(Ct, ncl, M.S.ml, M.cov, M.cnts + 3, 1);
        FL_LAUNCH_CHECK();
      }
      sweep_reset(c, M);
      const uint32_t ncov = read_u32(c, M.cnts + 3);
      // 4. facilities next to a covered client retire
      k_set_const_labels<<<(uint32_t)ceil_div(ncov ? ncov : 1, 256), 256, 0, c.s>>>(M.cov, ncov, M.lab, 0);
      FL_LAUNCH_CHECK();
      sweep(c, M, M.cov, ncov, R);
      k_collect_hit<<<(uint32_t)ceil_div(nr, 256), 256, 0, c.s>>>(M.act2, nr, M.S.ml, M.act, M.cnts + 4, 0);
      FL_LAUNCH_CHECK();
      sweep_reset(c, M);
      na = read_u32(c, M.cnts + 4);
    }
  }
  *rounds_out = total_rounds;
  return FL_OK;
}

}  // namespace fl
