// fl_ads.hip -- bottom-k all-distances sketches (ADS, Sec. 3.3) by rounds of
// edge relaxation on the GPU.
//
// Schedule.  Round D settles every sketch entry at distance exactly D (integer
// weights >= 1).  A candidate (r, D) reaches u from a neighbour v over an arc
// of weight w only if v inserted r in round D - w, so all entries at smaller
// distances are final when round D runs: sketches grow append-only, already in
// (distance, id) order, and no entry is ever evicted (the CleanUp of Alg. 2 is
// never needed).  With unit weights this is the superstep order of Alg. 2.
//
// Per round and vertex u (one wave64 per vertex):
//   1. stream the entries neighbours inserted at distance D - w (pull), drop
//      those whose rank is not below T_u, the k-th smallest rank of u's sketch
//      so far (k entries that all come first have a smaller rank), and those
//      already in u's bottom-k set (same vertex, shorter distance);
//   2. sort the survivors by vertex id in LDS (ties in distance go by id);
//   3. walk them in id order with the running bottom-k set in registers (one
//      rank per lane): a survivor enters iff fewer than k ranks of the set are
//      below it, and then joins the set;
//   4. append the accepted entries to u's sketch, record where they are for
//      the next rounds, and mark the neighbours that will have candidates.
// The running k-th smallest rank before each accepted entry is the HIP
// threshold T_j of that entry; it is stored for the estimator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fl_common.h"
#include "fl_ads.h"

namespace fl {

constexpr int ADS_WPB = 4;     // waves per block
constexpr uint32_t ADS_SB_MAX = 2048;  // largest survivor buffer per wave (ids; 4 waves fit 64 KB)

struct AdsArgs {
  uint32_t n, k, cap, W, NS, FW;
  PermKey rk;
  const uint64_t *row_ptr;
  const uint32_t *col;
  const uint32_t *w;
  uint32_t *sk_rank;
  uint32_t *sk_dist;
  uint32_t *thr;
  const uint32_t *thr_idx;  // nullptr: thr row = vertex
  uint32_t *bk;
  uint32_t *cnt;
  uint64_t *dinfo;
  uint32_t *flags;
  uint32_t *wl;
  uint32_t *wl_cnt;
  uint64_t *ctr;     // [64] relax_exec, [64] active vertices this round
  uint32_t *status;  // [0] capacity overflow, [1] survivor-buffer overflow
};

__device__ inline uint64_t pack_info(uint32_t round, uint32_t start, uint32_t count) {
  return ((uint64_t)round << 32) | ((uint64_t)start << 16) | (uint64_t)count;
}

// Append y to the worklist of slot s once (flag bit per (vertex, slot)).
// Lanes with want=false do nothing.  Aggregates the counter atomics per slot.
template <bool UNITW>
__device__ inline void mark_targets(const AdsArgs &P, bool want, uint32_t y, uint32_t s) {
  bool add = false;
  if (want) {
    uint32_t *word = &P.flags[(size_t)y * P.FW + (s >> 5)];
    const uint32_t bit = 1u << (s & 31);
    if (!(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
      add = !(atomicOr(word, bit) & bit);
  }
  uint64_t pend = __ballot(add);
  const int lane = lane_id();
  while (pend) {
    const int lead = __ffsll((long long)pend) - 1;
    const uint32_t sl = UNITW ? s : __shfl(s, lead, WAVE);
    const bool mine = add && (UNITW || s == sl);
    const uint64_t grp = __ballot(mine);
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(&P.wl_cnt[sl], (uint32_t)__popcll(grp));
    base = __shfl(base, lead, WAVE);
    if (mine) {
      P.wl[(size_t)sl * P.n + base + lanes_below(grp)] = y;
      add = false;
    }
    pend &= ~grp;
  }
}

template <bool UNITW>
__device__ inline void mark_neighbours(const AdsArgs &P, uint32_t u, uint32_t D) {
  const int lane = lane_id();
  const uint64_t a0 = P.row_ptr[u], a1 = P.row_ptr[u + 1];
  for (uint64_t b = a0; b < a1; b += WAVE) {
    const uint64_t a = b + lane;
    const bool valid = a < a1;
    uint32_t y = 0, s = 0;
    if (valid) {
      y = P.col[a];
      const uint32_t wv = UNITW ? 1u : P.w[a];
      s = (D + wv) % P.NS;
    }
    mark_targets<UNITW>(P, valid, y, s);
  }
}

// Round 0: every vertex holds (r(v), 0).  One wave per vertex.
template <bool UNITW>
__global__ __launch_bounds__(256) void k_ads_init(AdsArgs P, int mark) {
  const int lane = lane_id();
  const uint64_t u64 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (u64 >= P.n) return;
  const uint32_t u = (uint32_t)u64;
  const uint32_t r = perm_fwd(u, P.rk);
  if (lane == 0) {
    P.sk_rank[(size_t)u * P.cap] = r;
    P.sk_dist[(size_t)u * P.cap] = 0;
    if (P.thr) {
      const uint32_t ti = P.thr_idx ? P.thr_idx[u] : u;
      if (ti != INF32) P.thr[(size_t)ti * P.cap] = 0;
    }
    P.bk[(size_t)u * P.k] = r;
    P.cnt[u] = 1;
    P.dinfo[u] = pack_info(0, 0, 1);  // slot 0
  }
  if (mark) mark_neighbours<UNITW>(P, u, 0);
}

// Sort s_id[0..ns) ascending (bitonic over the next power of two <= SB).
__device__ inline void wave_sort_ids(uint32_t *s_id, uint32_t ns) {
  const int lane = lane_id();
  uint32_t p2 = 2;
  while (p2 < ns) p2 <<= 1;
  for (uint32_t i = ns + lane; i < p2; i += WAVE) s_id[i] = INF32;
  wave_lds_sync();
  for (uint32_t k2 = 2; k2 <= p2; k2 <<= 1) {
    for (uint32_t j = k2 >> 1; j > 0; j >>= 1) {
      for (uint32_t i = lane; i < p2; i += WAVE) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = s_id[i], b = s_id[ixj];
          const bool asc = (i & k2) == 0;
          if ((a > b) == asc) {
            s_id[i] = b;
            s_id[ixj] = a;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// Bottom-k pass over the id-sorted survivors (duplicates adjacent).  bkv/nb
// is the running set (one rank per lane, INF32 above nb).  Accepted ids are
// compacted to the front of s_id.  When thr_out is given, the HIP threshold
// of the i-th accepted entry goes to thr_out[i] (lane 0 writes; the caller
// guarantees room for `room` entries and the pass stops writing beyond it).
// Returns the number accepted.
__device__ inline uint32_t wave_bottomk_pass(uint32_t *s_id, uint32_t ns, uint32_t k, PermKey rk,
                                             uint32_t &bkv, uint32_t &nb, uint32_t *thr_out, uint32_t room) {
  const int lane = lane_id();
  uint32_t m = 0, prev = INF32;
  for (uint32_t i = 0; i < ns; ++i) {
    const uint32_t id = s_id[i];
    if (id == prev) continue;
    prev = id;
    const uint32_t r = perm_fwd(id, rk);
    const uint32_t below = (uint32_t)__popcll(__ballot(bkv < r));
    if (below < k) {
      const uint32_t Tj = nb < k ? 0u : __shfl(bkv, (int)k - 1, WAVE);
      const uint32_t up = __shfl_up(bkv, 1, WAVE);
      if ((uint32_t)lane > below && (uint32_t)lane < k) bkv = up;
      if ((uint32_t)lane == below) bkv = r;
      if (nb < k) ++nb;
      if (lane == 0) {
        s_id[m] = id;
        if (thr_out && m < room) thr_out[m] = Tj;
      }
      ++m;
    }
  }
  wave_lds_sync();
  return m;
}

template <bool UNITW>
__global__ __launch_bounds__(256) void k_ads_round(AdsArgs P, uint32_t D, const uint32_t *list,
                                                   uint32_t count, int sparse, int mark, uint32_t SB) {
  extern __shared__ uint32_t lds[];
  const int lane = lane_id();
  const int wv = threadIdx.x / WAVE;
  const uint64_t item = (uint64_t)blockIdx.x * ADS_WPB + wv;
  if (item >= count) return;
  uint32_t *s_bk = lds + wv * (SB + WAVE);
  uint32_t *s_id = s_bk + WAVE;

  const uint32_t u = list[item];
  const uint32_t slotD = D % P.NS;
  if (sparse && lane == 0)
    atomicAnd(&P.flags[(size_t)u * P.FW + (slotD >> 5)], ~(1u << (slotD & 31)));

  const uint32_t k = P.k;
  const uint32_t cu = P.cnt[u];
  uint32_t nb = cu < k ? cu : k;
  uint32_t bkv = (uint32_t)lane < nb ? P.bk[(size_t)u * k + lane] : INF32;
  s_bk[lane] = bkv;
  wave_lds_sync();
  const bool full = nb == k;
  const uint32_t T = full ? __shfl(bkv, (int)k - 1, WAVE) : INF32;
  const uint32_t nb0 = nb;
  const uint32_t bkv0 = bkv;

  uint32_t ns = 0;
  uint64_t examined = 0;
  const uint64_t a0 = P.row_ptr[u], a1 = P.row_ptr[u + 1];
  for (uint64_t b = a0; b < a1; b += WAVE) {
    const uint64_t a = b + lane;
    uint32_t v = 0, st = 0, cn = 0;
    if (a < a1) {
      v = P.col[a];
      const uint32_t wv_ = UNITW ? 1u : P.w[a];
      if (wv_ <= D) {
        const uint32_t src = D - wv_;
        const uint64_t info = P.dinfo[(size_t)(src % P.NS) * P.n + v];
        if ((uint32_t)(info >> 32) == src) {
          st = (uint32_t)(info >> 16) & 0xFFFFu;
          cn = (uint32_t)info & 0xFFFFu;
        }
      }
    }
    const uint32_t incl = wave_scan_incl(cn);
    const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
    const uint32_t excl = incl - cn;
    examined += total;
    for (uint32_t c0 = 0; c0 < total; c0 += WAVE) {
      const uint32_t idx = c0 + lane;
      // owner lane: first lane whose inclusive count exceeds idx
      uint32_t pos = 0;
#pragma unroll
      for (uint32_t s = 32; s >= 1; s >>= 1) {
        const uint32_t val = __shfl(incl, (int)(pos + s - 1), WAVE);
        if (val <= idx) pos += s;
      }
      const bool valid = idx < total;
      const uint32_t ov = __shfl(v, (int)pos, WAVE);
      const uint32_t ost = __shfl(st, (int)pos, WAVE);
      const uint32_t oex = __shfl(excl, (int)pos, WAVE);
      uint32_t r = INF32;
      if (valid) r = P.sk_rank[(size_t)ov * P.cap + ost + (idx - oex)];
      bool pass = valid && (!full || r < T);
      if (pass) {
        // already in the bottom-k set?  (binary search in the sorted set)
        uint32_t lo = 0, hi = nb0;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_bk[mid] < r) lo = mid + 1;
          else hi = mid;
        }
        if (lo < nb0 && s_bk[lo] == r) pass = false;
      }
      uint64_t msk = __ballot(pass);
      if (msk) {
        const uint32_t np = (uint32_t)__popcll(msk);
        if (ns + np > SB) {
          // shrink the buffer: keep what survives against the current set
          wave_sort_ids(s_id, ns);
          uint32_t tb = bkv0, tn = nb0;
          ns = wave_bottomk_pass(s_id, ns, k, P.rk, tb, tn, nullptr, 0);
          if (ns + np > SB) {
            if (lane == 0) atomicOr(&P.status[1], 1u);
            return;
          }
        }
        if (pass) s_id[ns + lanes_below(msk)] = perm_inv(r, P.rk);
        ns += np;
        wave_lds_sync();
      }
    }
  }
  if (lane == 0) atomicAdd((unsigned long long *)&P.ctr[blockIdx.x & 63], (unsigned long long)examined);
  if (ns == 0) return;

  wave_sort_ids(s_id, ns);
  const uint32_t ti = P.thr ? (P.thr_idx ? P.thr_idx[u] : u) : INF32;
  uint32_t *thr_out = ti != INF32 ? P.thr + (size_t)ti * P.cap + cu : nullptr;
  const uint32_t m = wave_bottomk_pass(s_id, ns, k, P.rk, bkv, nb, thr_out, P.cap - cu);
  if (m == 0) return;
  if (cu + m > P.cap) {
    if (lane == 0) atomicOr(&P.status[0], 1u);
    return;
  }
  const size_t base = (size_t)u * P.cap + cu;
  for (uint32_t i = lane; i < m; i += WAVE) {
    P.sk_rank[base + i] = perm_fwd(s_id[i], P.rk);
    P.sk_dist[base + i] = D;
  }
  if ((uint32_t)lane < nb) P.bk[(size_t)u * k + lane] = bkv;
  if (lane == 0) {
    P.cnt[u] = cu + m;
    P.dinfo[(size_t)slotD * P.n + u] = pack_info(D, cu, m);
    atomicAdd((unsigned long long *)&P.ctr[64 + (blockIdx.x & 63)], 1ull);
  }
  if (mark) mark_neighbours<UNITW>(P, u, D);
}

// list of vertices with at least one arc, hubs first is not needed: any order
__global__ void k_nonisolated_flags(uint32_t n, const uint64_t *row_ptr, uint32_t *flag) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = row_ptr[i + 1] > row_ptr[i] ? 1u : 0u;
}
__global__ void k_compact(uint32_t n, const uint32_t *flag, const uint64_t *pos, uint32_t *out) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (uint32_t)i;
}

// Compact the per-vertex sketches into CSR (one wave per vertex).
__global__ __launch_bounds__(256) void k_ads_export(uint32_t n, uint32_t cap, const uint32_t *cnt,
                                                    const uint64_t *off, const uint32_t *sk_rank,
                                                    const uint32_t *sk_dist, const uint32_t *thr,
                                                    uint32_t *o_rank, uint32_t *o_dist, uint32_t *o_thr) {
  const uint64_t u = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (u >= n) return;
  const uint32_t c = cnt[u];
  const uint64_t o = off[u];
  for (uint32_t i = lane_id(); i < c; i += WAVE) {
    o_rank[o + i] = sk_rank[u * cap + i];
    o_dist[o + i] = sk_dist[u * cap + i];
    o_thr[o + i] = thr[u * cap + i];
  }
}

uint32_t ads_capacity(uint32_t n, uint32_t k) {
  double lnr = std::log((double)n / (double)k);
  if (lnr < 0) lnr = 0;
  double mean = (double)k * (1.0 + lnr);
  double sd = std::sqrt((double)k * lnr + 1.0);
  double cap = std::ceil(mean + 8.0 * sd + 16.0);
  uint64_t c = ((uint64_t)cap + 15) & ~15ull;
  if (c > n) c = n;
  if (c < 1) c = 1;
  return (uint32_t)c;
}

// Builds the sketches.  Returns FL_OK, or FL_ENOMEM / FL_ENOTIMPL.  The
// caller provides cap; on capacity overflow the call reports *need_more.
static int ads_run(Ctx &c, const Graph &g, const AdsConfig &cfg, AdsOut &o, bool *need_more) {
  const uint32_t n = g.n, k = cfg.k, cap = o.cap;
  const uint32_t W = g.w ? g.max_w : 1u;
  const uint32_t NS = W + 1;
  const uint32_t FW = (NS + 31) / 32;
  const bool unit = g.w == nullptr;
  *need_more = false;

  AdsArgs P{};
  P.n = n;
  P.k = k;
  P.cap = cap;
  P.W = W;
  P.NS = NS;
  P.FW = FW;
  P.rk = perm_key(cfg.seed, 1);
  P.row_ptr = g.row_ptr;
  P.col = g.col;
  P.w = g.w;
  P.sk_rank = o.sk_rank;
  P.sk_dist = o.sk_dist;
  P.thr = o.thr;
  P.thr_idx = o.thr_idx;
  P.bk = c.arena->get<uint32_t>((size_t)n * k);
  P.cnt = o.cnt;
  P.dinfo = c.arena->get<uint64_t>((size_t)NS * n);
  P.flags = c.arena->get<uint32_t>((size_t)n * FW);
  P.wl = c.arena->get<uint32_t>((size_t)NS * n);
  P.wl_cnt = c.arena->get<uint32_t>(NS);
  P.ctr = c.arena->get<uint64_t>(128);
  P.status = c.arena->get<uint32_t>(4);
  fill_u64(c, P.dinfo, (size_t)NS * n, INF64);
  fill_u32(c, P.flags, (size_t)n * FW, 0);
  fill_u32(c, P.wl_cnt, NS, 0);
  fill_u64(c, P.ctr, 128, 0);
  fill_u32(c, P.status, 4, 0);

  // dense list: vertices with at least one arc
  uint32_t *dense = nullptr;
  uint32_t n_dense = 0;
  const bool dense_ok = unit && !(cfg.flags & FL_FLAG_NO_DENSE);
  if (dense_ok) {
    uint32_t *fl = c.arena->get<uint32_t>(n);
    uint64_t *pos = c.arena->get<uint64_t>((size_t)n + 1);
    dense = c.arena->get<uint32_t>(n);
    k_nonisolated_flags<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, g.row_ptr, fl);
    FL_LAUNCH_CHECK();
    scan_u32_to_u64(c, fl, pos, n);
    k_compact<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, fl, pos, dense);
    FL_LAUNCH_CHECK();
    FL_HIP(hipMemcpyAsync(c.h_status, pos + n, 8, hipMemcpyDeviceToHost, c.s));
    c.sync();
    n_dense = (uint32_t)c.h_status[0];
  }
  const uint64_t dense_threshold = (uint64_t)n_dense / 32;

  // round 0
  bool mark = !dense_ok || n_dense <= dense_threshold;
  {
    uint64_t blocks = ceil_div((uint64_t)n * WAVE, 256);
    if (unit) k_ads_init<true><<<(uint32_t)blocks, 256, 0, c.s>>>(P, mark ? 1 : 0);
    else k_ads_init<false><<<(uint32_t)blocks, 256, 0, c.s>>>(P, mark ? 1 : 0);
    FL_LAUNCH_CHECK();
  }
  bool sparse = mark;  // mode of round 1
  // survivor buffer: a whole distance level of one sketch (at most cap
  // entries) plus one chunk of candidates fits
  uint32_t SB = 256;
  while (SB < cap + WAVE && SB < ADS_SB_MAX) SB <<= 1;
  const size_t lds_bytes = (size_t)ADS_WPB * (SB + WAVE) * sizeof(uint32_t);
  hipEvent_t e0, e1;
  FL_HIP(hipEventCreate(&e0));
  FL_HIP(hipEventCreate(&e1));
  struct EvDel {
    hipEvent_t a, b;
    ~EvDel() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evdel{e0, e1};
  o.kernel_ms = 0.0;
  o.launches = 0;
  uint64_t active_prev = n;
  uint32_t rounds = 0;
  std::vector<uint32_t> hwl(NS);
  for (uint32_t D = 1;; ++D) {
    const uint32_t slot = D % NS;
    // worklist size of this round
    uint32_t count;
    const uint32_t *list;
    if (sparse) {
      FL_HIP(hipMemcpyAsync(c.h_status, P.wl_cnt + slot, 4, hipMemcpyDeviceToHost, c.s));
      c.sync();
      count = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
      list = P.wl + (size_t)slot * n;
    } else {
      count = n_dense;
      list = dense;
    }
    // marking decision for this round (decides the mode of the next one)
    mark = !dense_ok || active_prev <= dense_threshold;
    fill_u64(c, P.ctr + 64, 64, 0);
    if (count) {
      const uint64_t blocks = ceil_div(count, ADS_WPB);
      FL_HIP(hipEventRecord(e0, c.s));
      if (unit)
        k_ads_round<true><<<(uint32_t)blocks, 256, lds_bytes, c.s>>>(P, D, list, count, sparse ? 1 : 0,
                                                                     mark ? 1 : 0, SB);
      else
        k_ads_round<false><<<(uint32_t)blocks, 256, lds_bytes, c.s>>>(P, D, list, count, sparse ? 1 : 0,
                                                                      mark ? 1 : 0, SB);
      FL_LAUNCH_CHECK();
      FL_HIP(hipEventRecord(e1, c.s));
    }
    if (sparse) fill_u32(c, P.wl_cnt + slot, 1, 0);
    ++rounds;
    // status: overflow flags, active count, pending worklists
    static_assert(sizeof(uint64_t) * 64 <= 4096 * 8, "status");
    FL_HIP(hipMemcpyAsync(c.h_status, P.status, 8, hipMemcpyDeviceToHost, c.s));
    FL_HIP(hipMemcpyAsync(c.h_status + 1, P.ctr + 64, 64 * 8, hipMemcpyDeviceToHost, c.s));
    FL_HIP(hipMemcpyAsync(hwl.data(), P.wl_cnt, NS * 4, hipMemcpyDeviceToHost, c.s));
    c.sync();
    if (count) {
      float ms = 0.f;
      FL_HIP(hipEventElapsedTime(&ms, e0, e1));
      o.kernel_ms += ms;
      o.launches += 1;
    }
    const uint32_t st0 = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
    const uint32_t st1 = (uint32_t)(c.h_status[0] >> 32);
    if (st0) {
      *need_more = true;
      return FL_OK;
    }
    if (st1) return FL_ENOMEM;
    uint64_t active = 0;
    for (int i = 0; i < 64; ++i) active += c.h_status[1 + i];
    uint64_t pending = 0;
    for (uint32_t s = 0; s < NS; ++s) pending += hwl[s];
    if (unit) {
      if (active == 0) break;
    } else {
      if (pending == 0) break;
    }
    active_prev = active;
    sparse = mark;
    // a settled entry is at most (n-1) max_w away: more rounds mean a bug
    if ((uint64_t)D > (uint64_t)(n - 1) * W + 2) return FL_EHIP;
  }
  o.rounds = rounds;
  std::vector<uint64_t> hc(64);
  FL_HIP(hipMemcpyAsync(hc.data(), P.ctr, 64 * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  o.relax_exec = 0;
  for (int i = 0; i < 64; ++i) o.relax_exec += hc[i];
  return FL_OK;
}

int ads_build(Ctx &c, const Graph &g, const AdsConfig &cfg, AdsOut &o) {
  if (cfg.k == 0) return FL_EINVAL;
  if (cfg.k > MAX_K) return FL_ENOTIMPL;
  if (g.w && g.max_w > MAX_W) return FL_ENOTIMPL;
  uint32_t cap = ads_capacity(g.n, cfg.k);
  for (int attempt = 0; attempt < 6; ++attempt) {
    if (cap > MAX_CAP) return FL_ENOTIMPL;
    const size_t mark = c.arena->used();
    o.cap = cap;
    o.sk_rank = c.arena->get<uint32_t>((size_t)g.n * cap);
    o.sk_dist = c.arena->get<uint32_t>((size_t)g.n * cap);
    o.cnt = c.arena->get<uint32_t>(g.n);
    const uint32_t thr_rows = cfg.thr_rows;
    o.thr = thr_rows ? c.arena->get<uint32_t>((size_t)thr_rows * cap) : nullptr;
    o.thr_idx = cfg.thr_idx;
    const size_t after_out = c.arena->used();
    bool more = false;
    int rc = ads_run(c, g, cfg, o, &more);
    if (rc != FL_OK) return rc;
    // scratch of the run is no longer needed; keep the outputs
    (void)mark;
    c.arena->rewind(after_out);
    if (std::getenv("FL_DEBUG"))
      std::fprintf(stderr, "[fl] sketches: cap %u rounds %u overflow %d\n", cap, o.rounds, (int)more);
    if (!more) return FL_OK;
    uint64_t nc = (uint64_t)cap * 3 / 2 + 16;
    if (nc > g.n) nc = g.n;
    if (nc == cap) return FL_ENOMEM;
    c.arena->rewind(mark);
    cap = (uint32_t)nc;
  }
  return FL_ENOMEM;
}

int ads_export(Ctx &c, const Graph &g, const AdsOut &o, uint64_t *off, uint32_t *rank, uint32_t *dist,
               uint32_t *thr) {
  k_ads_export<<<(uint32_t)ceil_div((uint64_t)g.n * WAVE, 256), 256, 0, c.s>>>(
      g.n, o.cap, o.cnt, off, o.sk_rank, o.sk_dist, o.thr, rank, dist, thr);
  FL_LAUNCH_CHECK();
  return FL_OK;
}

}  // namespace fl
