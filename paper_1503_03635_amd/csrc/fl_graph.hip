// fl_graph.hip -- graph-level kernels: input validation, fills, scans,
// reductions, and the frontier Bellman-Ford used for the multi-source
// shortest-path sweeps (gamma, distance to the open set, assignment).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "fl_common.h"
#include "fl_frontier.h"

namespace fl {

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *p, uint64_t n, T v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
template <class T>
static void fill_t(Ctx &c, T *p, uint64_t n, T v) {
  if (n == 0) return;
  uint64_t blocks = ceil_div(n, 256);
  if (blocks > 65536) blocks = 65536;
  k_fill<T><<<(uint32_t)blocks, 256, 0, c.s>>>(p, n, v);
  FL_LAUNCH_CHECK();
}
void fill_u32(Ctx &c, uint32_t *p, uint64_t n, uint32_t v) { fill_t(c, p, n, v); }
void fill_u64(Ctx &c, uint64_t *p, uint64_t n, uint64_t v) { fill_t(c, p, n, v); }
void fill_u8(Ctx &c, uint8_t *p, uint64_t n, uint8_t v) { fill_t(c, p, n, v); }
void fill_f64(Ctx &c, double *p, uint64_t n, double v) { fill_t(c, p, n, v); }

// ---------------------------------------------------------------------------
// Validation (a simple undirected graph as a symmetric CSR, Sec. 3.1; a
// directed graph gives its out-arcs and skips the symmetry test).  One wave
// per vertex (waves stride over the vertices); lanes walk the row.  err
// bits: 1 = structural error.  Also reduces max weight and max facility
// cost.  Each block reduces its waves' results in LDS and adds them to
// stripe blockIdx.x % stripes, one 128-byte line per stripe: v32[32 s + 0]
// error bits, [32 s + 1] max weight, [32 s + 2] max cost; lt[16 s + 0]
// leading arcs, [16 s + 1] trailing arcs.
//
// Symmetry: an arc u -> v is "leading" when u has the larger degree (ties:
// the larger id).  Only leading arcs look up their reverse, by binary search
// in the row of the smaller end, and must find it with the same weight; the
// leading and trailing arcs are counted.  The reverse of a leading arc is a
// trailing arc, distinct arcs have distinct reverses, so equal counts mean
// every trailing arc is the reverse of a leading one: the arc set is
// symmetric with equal weights.
// ---------------------------------------------------------------------------
__device__ inline bool find_arc(const uint64_t *row_ptr, const uint32_t *col, uint64_t m, uint32_t u,
                                uint32_t v, uint64_t *pos) {
  uint64_t lo = row_ptr[u], hi = row_ptr[u + 1];
  const uint64_t end = hi;
  if (hi > m || lo > hi) return false;  // malformed row: never read past col[m-1]
  while (lo < hi) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  *pos = lo;
  return lo < end && col[lo] == v;
}

constexpr uint32_t VAL_STRIDE32 = 32, VAL_STRIDE64 = 16;  // one 128-byte line per stripe
constexpr uint32_t VAL_BLOCKS = 4096;                      // grid of a validation launch (at most)
__global__ __launch_bounds__(256) void k_validate(uint32_t n, uint64_t m, const uint64_t *row_ptr,
                                                  const uint32_t *col, const uint32_t *w,
                                                  const uint32_t *fac_cost, uint32_t *v32, uint32_t stripes,
                                                  uint32_t directed, unsigned long long *lt) {
  __shared__ uint32_t sh_bad[256 / WAVE], sh_mw[256 / WAVE], sh_mc[256 / WAVE];
  __shared__ unsigned long long sh_lead[256 / WAVE], sh_trail[256 / WAVE];
  const int lane = lane_id();
  const uint32_t wv = threadIdx.x / WAVE;
  uint32_t bad = 0, mw = 0, mc = 0;
  uint64_t nlead = 0, ntrail = 0;
  const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x / WAVE);
  for (uint64_t u64 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; u64 < n; u64 += nwaves) {
    const uint32_t u = (uint32_t)u64;
    const uint64_t a0 = row_ptr[u], a1 = row_ptr[u + 1];
    if (a1 < a0 || a1 > m) {
      bad = 1;
      continue;
    }
    const uint64_t du = a1 - a0;
    for (uint64_t a = a0 + lane; a < a1; a += WAVE) {
      uint32_t v = col[a];
      uint32_t wv_ = w ? w[a] : 1u;
      if (v >= n || v == u || wv_ == 0) { bad = 1; continue; }
      if (a > a0 && col[a - 1] >= v) { bad = 1; continue; }
      if (!directed) {
        const uint64_t b0 = row_ptr[v], b1 = row_ptr[v + 1];
        if (b1 < b0 || b1 > m) { bad = 1; continue; }
        const uint64_t dv = b1 - b0;
        if (du > dv || (du == dv && u > v)) {
          ++nlead;
          uint64_t back;
          if (!find_arc(row_ptr, col, m, v, u, &back)) { bad = 1; continue; }
          if ((w ? w[back] : 1u) != wv_) bad = 1;
        } else {
          ++ntrail;
        }
      }
      mw = wv_ > mw ? wv_ : mw;
    }
    if (fac_cost && lane == 0) {
      const uint32_t cst = fac_cost[u];
      if (cst != FL_NOT_FACILITY && cst > mc) mc = cst;
    }
  }
  const uint64_t anybad = __ballot(bad != 0);
  mw = ~wave_min_u32(~mw);  // wave max
  mc = ~wave_min_u32(~mc);
  const uint64_t lead = wave_sum_u64(nlead), trail = wave_sum_u64(ntrail);
  if (lane == 0) {
    sh_bad[wv] = anybad ? 1u : 0u;
    sh_mw[wv] = mw;
    sh_mc[wv] = mc;
    sh_lead[wv] = lead;
    sh_trail[wv] = trail;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = 0, x = 0, c = 0;
    unsigned long long l = 0, t = 0;
    for (uint32_t i = 0; i < blockDim.x / WAVE; ++i) {
      b |= sh_bad[i];
      x = sh_mw[i] > x ? sh_mw[i] : x;
      c = sh_mc[i] > c ? sh_mc[i] : c;
      l += sh_lead[i];
      t += sh_trail[i];
    }
    const uint32_t st = blockIdx.x % stripes;
    uint32_t *q = v32 + (size_t)st * VAL_STRIDE32;
    unsigned long long *r = lt + (size_t)st * VAL_STRIDE64;
    if (b) atomicOr(&q[0], 1u);
    if (x) atomicMax(&q[1], x);
    if (c) atomicMax(&q[2], c);
    if (l) atomicAdd(&r[0], l);
    if (t) atomicAdd(&r[1], t);
  }
}

static uint32_t validate_blocks(uint32_t n) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(ceil_div((uint64_t)n * WAVE, 256), VAL_BLOCKS));
}

int validate_graph(Ctx &c, const fl_problem *p, bool directed, uint32_t *max_w_out, uint32_t *max_cost_out) {
  const uint32_t n = p->n;
  // row_ptr[0] and row_ptr[n]
  uint64_t ends[2];
  FL_HIP(hipMemcpyAsync(&ends[0], p->row_ptr, 8, hipMemcpyDeviceToHost, c.s));
  FL_HIP(hipMemcpyAsync(&ends[1], p->row_ptr + n, 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  if (ends[0] != 0 || ends[1] != p->n_arcs) return FL_EINVAL;
  constexpr uint32_t S = 64;  // stripes
  uint32_t *d = c.arena->get<uint32_t>((size_t)S * VAL_STRIDE32);
  uint64_t *lt = c.arena->get<uint64_t>((size_t)S * VAL_STRIDE64);
  fill_u32(c, d, (size_t)S * VAL_STRIDE32, 0);
  fill_u64(c, lt, (size_t)S * VAL_STRIDE64, 0);
  k_validate<<<validate_blocks(n), 256, 0, c.s>>>(n, p->n_arcs, p->row_ptr, p->col, p->w, p->fac_cost, d, S,
                                                  directed ? 1u : 0u, reinterpret_cast<unsigned long long *>(lt));
  FL_LAUNCH_CHECK();
  std::vector<uint32_t> h((size_t)S * VAL_STRIDE32);
  std::vector<uint64_t> hl((size_t)S * VAL_STRIDE64);
  FL_HIP(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, c.s));
  FL_HIP(hipMemcpyAsync(hl.data(), lt, hl.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  uint32_t err = 0, mw = 1, mc = 0;
  uint64_t lead = 0, trail = 0;
  for (uint32_t i = 0; i < S; ++i) {
    const uint32_t *q = &h[(size_t)i * VAL_STRIDE32];
    err |= q[0];
    mw = q[1] > mw ? q[1] : mw;
    mc = q[2] > mc ? q[2] : mc;
    lead += hl[(size_t)i * VAL_STRIDE64];
    trail += hl[(size_t)i * VAL_STRIDE64 + 1];
  }
  if (err || lead != trail) return FL_EINVAL;
  *max_w_out = mw;
  *max_cost_out = mc;
  return FL_OK;
}

// row_ptr[0] == 0 and row_ptr[n] == n_arcs of each graph
struct EndsDesc {
  const uint64_t *row_ptr;
  uint32_t n;
  uint64_t m;
};
__global__ void k_check_ends(const EndsDesc *d, uint32_t G, uint32_t *err) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G && (d[g].row_ptr[0] != 0 || d[g].row_ptr[d[g].n] != d[g].m)) err[(size_t)g * VAL_STRIDE32] |= 2u;
}

void validate_graphs(Ctx &c, const fl_problem *const *ps, uint32_t G, bool directed, std::vector<int> &rc,
                     std::vector<uint32_t> &max_w, std::vector<uint32_t> &max_cost) {
  // one stripe (a 128-byte line of counters) per graph
  uint32_t *d = c.arena->get<uint32_t>((size_t)VAL_STRIDE32 * G);
  uint64_t *lt = c.arena->get<uint64_t>((size_t)VAL_STRIDE64 * G);
  fill_u64(c, lt, (size_t)VAL_STRIDE64 * G, 0);
  EndsDesc *ed = c.arena->get<EndsDesc>(G);
  std::vector<EndsDesc> hd(G);
  for (uint32_t g = 0; g < G; ++g) hd[g] = EndsDesc{ps[g]->row_ptr, ps[g]->n, ps[g]->n_arcs};
  fill_u32(c, d, (size_t)VAL_STRIDE32 * G, 0);
  FL_HIP(hipMemcpyAsync(ed, hd.data(), G * sizeof(EndsDesc), hipMemcpyHostToDevice, c.s));
  k_check_ends<<<(uint32_t)ceil_div(G, 256), 256, 0, c.s>>>(ed, G, d);
  FL_LAUNCH_CHECK();
  // the row checks read row_ptr only inside [0, n_arcs], whatever its values
  for (uint32_t g = 0; g < G; ++g) {
    const fl_problem *p = ps[g];
    k_validate<<<validate_blocks(p->n), 256, 0, c.s>>>(p->n, p->n_arcs, p->row_ptr, p->col, p->w, p->fac_cost,
                                                       d + (size_t)VAL_STRIDE32 * g, 1, directed ? 1u : 0u,
                                                       reinterpret_cast<unsigned long long *>(lt) +
                                                           (size_t)VAL_STRIDE64 * g);
    FL_LAUNCH_CHECK();
  }
  std::vector<uint32_t> h((size_t)VAL_STRIDE32 * G);
  std::vector<uint64_t> hl((size_t)VAL_STRIDE64 * G);
  FL_HIP(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, c.s));
  FL_HIP(hipMemcpyAsync(hl.data(), lt, hl.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  rc.assign(G, FL_OK);
  max_w.assign(G, 1);
  max_cost.assign(G, 0);
  for (uint32_t g = 0; g < G; ++g) {
    const uint32_t *q = &h[(size_t)VAL_STRIDE32 * g];
    const uint64_t *r = &hl[(size_t)VAL_STRIDE64 * g];
    if (q[0] || r[0] != r[1]) rc[g] = FL_EINVAL;
    max_w[g] = q[1] > 1 ? q[1] : 1u;
    max_cost[g] = q[2];
  }
}

std::vector<uint64_t> read_seg_ctr(Ctx &c, const uint64_t *d, uint32_t G, uint32_t nf, uint32_t stripes,
                                   bool max_last) {
  std::vector<uint64_t> h((size_t)G * nf * stripes);
  FL_HIP(hipMemcpyAsync(h.data(), d, h.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  std::vector<uint64_t> out((size_t)G * nf, 0);
  for (size_t i = 0; i < out.size(); ++i) {
    const bool mx = max_last && (i % nf) == nf - 1;
    for (uint32_t s = 0; s < stripes; ++s) {
      const uint64_t x = h[i * stripes + s];
      out[i] = mx ? (x > out[i] ? x : out[i]) : out[i] + x;
    }
  }
  return out;
}

// ---------------------------------------------------------------------------
// Exclusive scan u32 -> u64 (n+1 outputs).  Three passes: per-block sums,
// one block scans the block sums, blocks add their prefix.
// ---------------------------------------------------------------------------
constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr uint32_t SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

__device__ inline uint64_t block_scan_excl_u64(uint64_t x, uint64_t *tmp, uint64_t *total) {
  // wave-level inclusive scan then block combine
  const int lane = lane_id(), wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  uint64_t inc = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint64_t y = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += y;
  }
  if (lane == WAVE - 1) tmp[wv] = inc;
  __syncthreads();
  if (wv == 0) {
    uint64_t t = lane < nw ? tmp[lane] : 0;
    uint64_t ti = t;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
      uint64_t y = __shfl_up(ti, d, WAVE);
      if (lane >= d) ti += y;
    }
    if (lane < nw) tmp[lane] = ti - t;
    if (lane == nw - 1) tmp[WAVE] = ti;
  }
  __syncthreads();
  uint64_t r = tmp[wv] + inc - x;
  *total = tmp[WAVE];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const uint32_t *in, uint32_t n, uint64_t *out,
                                                          uint64_t *tile_sums) {
  __shared__ uint64_t tmp[WAVE + 1];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint64_t total;
  uint64_t pre = block_scan_excl_u64(s, tmp, &total);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = pre;
    pre += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(uint64_t *sums, uint32_t count, uint64_t *grand) {
  __shared__ uint64_t tmp[WAVE + 1];
  uint64_t carry = 0;
  for (uint32_t base = 0; base < count; base += SCAN_BLOCK) {
    uint32_t i = base + threadIdx.x;
    uint64_t x = i < count ? sums[i] : 0;
    uint64_t total;
    uint64_t pre = block_scan_excl_u64(x, tmp, &total);
    if (i < count) sums[i] = pre + carry;
    carry += total;
  }
  if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_add(uint64_t *out, uint32_t n, const uint64_t *sums) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  const uint64_t add = sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) out[base + i] += add;
}

size_t scan_sums_count(uint32_t n) { return ceil_div(n ? n : 1, SCAN_TILE) + 1; }

void scan_u32_to_u64(Ctx &c, const uint32_t *in, uint64_t *out, uint32_t n, uint64_t *sums) {
  uint32_t tiles = (uint32_t)ceil_div(n ? n : 1, SCAN_TILE);
  if (!sums) sums = c.arena->get<uint64_t>(tiles + 1);
  k_scan_tiles<<<tiles, SCAN_BLOCK, 0, c.s>>>(in, n, out, sums);
  FL_LAUNCH_CHECK();
  k_scan_sums<<<1, SCAN_BLOCK, 0, c.s>>>(sums, tiles, out + n);
  FL_LAUNCH_CHECK();
  k_scan_add<<<tiles, SCAN_BLOCK, 0, c.s>>>(out, n, sums);
  FL_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// In-arcs of a directed graph (Sec. 3.1 admits directed graphs): a counting
// sort of the arcs by head.  Within a row the order is that of the atomic
// cursor; nothing downstream depends on it (sketches, labels and sweeps are
// minima over the row).
// ---------------------------------------------------------------------------
__global__ void k_in_degree(uint64_t m, const uint32_t *col, uint32_t *deg) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m; a += stride) atomicAdd(&deg[col[a]], 1u);
}

// row_ptr is validated: row_ptr[0] = 0, non-decreasing, row_ptr[n] = m, and
// every col < n, so the tail search stays in [0, n) and p < in_ptr[v + 1].
__global__ void k_in_scatter(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                             const uint32_t *w, const uint64_t *in_ptr, uint32_t *cur, uint32_t *in_col,
                             uint32_t *in_w, uint32_t *out_to_in) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m; a += stride) {
    uint32_t lo = 0, hi = n;  // row_ptr[lo] <= a < row_ptr[hi]
    while (hi - lo > 1) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (row_ptr[mid] <= a) lo = mid;
      else hi = mid;
    }
    const uint32_t v = col[a];
    const uint64_t p = in_ptr[v] + atomicAdd(&cur[v], 1u);
    in_col[p] = lo;
    if (w) in_w[p] = w[a];
    if (out_to_in) out_to_in[a] = (uint32_t)p;
  }
}

size_t transpose_bytes(uint32_t n, uint64_t m, bool weighted) {
  return (size_t)(n + 1) * 8 + (size_t)n * 4 + (size_t)m * (weighted ? 12 : 8) + ((size_t)1 << 20);
}

void set_in_arcs(Ctx &c, Graph &g, bool directed) {
  if (!directed) {
    g.in_ptr = g.row_ptr;
    g.in_col = g.col;
    g.in_w = g.w;
    return;
  }
  const uint32_t n = g.n;
  const uint64_t m = g.m;
  uint32_t *deg = c.arena->get<uint32_t>(n);
  uint64_t *ip = c.arena->get<uint64_t>((size_t)n + 1);
  uint32_t *ic = c.arena->get<uint32_t>(m ? m : 1);
  uint32_t *iw = g.w ? c.arena->get<uint32_t>(m ? m : 1) : nullptr;
  // arc positions fit 32 bits below 2^32 arcs; beyond, the sketch rounds scan every in-arc
  uint32_t *o2i = m < 0xFFFFFFFFull ? c.arena->get<uint32_t>(m ? m : 1) : nullptr;
  fill_u32(c, deg, n, 0);
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(ceil_div(m ? m : 1, 256), 16384);
  if (m) {
    k_in_degree<<<blocks, 256, 0, c.s>>>(m, g.col, deg);
    FL_LAUNCH_CHECK();
  }
  scan_u32_to_u64(c, deg, ip, n);
  fill_u32(c, deg, n, 0);  // now the per-row cursor
  if (m) {
    k_in_scatter<<<blocks, 256, 0, c.s>>>(n, m, g.row_ptr, g.col, g.w, ip, deg, ic, iw, o2i);
    FL_LAUNCH_CHECK();
  }
  g.in_ptr = ip;
  g.in_col = ic;
  g.in_w = iw;
  g.out_to_in = o2i;
}

// ---------------------------------------------------------------------------
// sum_v cnt[v] * deg(v) and sum_v cnt[v]
// ---------------------------------------------------------------------------
__global__ void k_ads_totals(uint32_t n, const uint64_t *row_ptr, const uint32_t *cnt, const uint32_t *gid,
                             uint64_t *ctr, uint32_t stripes) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  uint64_t r = 0, e = 0;
  uint32_t g = 0;
  if (valid) {
    e = cnt[i];
    r = e * (row_ptr[i + 1] - row_ptr[i]);
    g = seg_of(gid, (uint32_t)i);
  }
  seg_add((unsigned long long *)ctr, valid, g, 0, 2, stripes, r);
  seg_add((unsigned long long *)ctr, valid, g, 1, 2, stripes, e);
}

void ads_totals(Ctx &c, const Graph &g, const uint32_t *gid, uint32_t G, const uint32_t *cnt,
                std::vector<uint64_t> &relax_alg, std::vector<uint64_t> &entries) {
  const uint32_t stripes = G == 1 ? 64 : 1;
  uint64_t *ctr = c.arena->get<uint64_t>((size_t)2 * G * stripes);
  fill_u64(c, ctr, (size_t)2 * G * stripes, 0);
  k_ads_totals<<<(uint32_t)ceil_div(g.n, 256), 256, 0, c.s>>>(g.n, g.row_ptr, cnt, gid, ctr, stripes);
  FL_LAUNCH_CHECK();
  const std::vector<uint64_t> h = read_seg_ctr(c, ctr, G, 2, stripes);
  relax_alg.resize(G);
  entries.resize(G);
  for (uint32_t q = 0; q < G; ++q) {
    relax_alg[q] = h[2 * q];
    entries[q] = h[2 * q + 1];
  }
}

// ---------------------------------------------------------------------------
// Frontier Bellman-Ford on packed labels (value << 32 | tie): a label moves
// along an arc of weight w as label + (w << 32).  Each vertex of the current
// frontier pushes its label to all neighbours with 64-bit atomicMin; a
// neighbour whose label dropped joins the next frontier once (stamped with
// the iteration number).  The fixed point is the lexicographic minimum over
// sources of (init value + distance, tie).
// ---------------------------------------------------------------------------
// Appends to the next frontier, staged per wave in LDS (2 WAVE entries) and
// written WAVE at a time with one atomic: every wave of a large frontier
// appends at nearly every step, and per-step atomics queue on the one count.
struct WaveQ {
  uint32_t *buf;  // this wave's LDS staging area
  uint32_t cnt;   // staged entries (wave-uniform, < WAVE between calls)
  uint32_t *next, *nnext;
};

// every lane calls, converged
__device__ inline void wq_push(WaveQ &q, bool add, uint32_t y) {
  const int lane = lane_id();
  const uint64_t m = __ballot(add);
  if (!m) return;
  if (add) q.buf[q.cnt + lanes_below(m)] = y;
  q.cnt += (uint32_t)__popcll(m);
  if (q.cnt < (uint32_t)WAVE) return;
  wave_lds_sync();
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(q.nnext, (uint32_t)WAVE);
  base = __shfl(base, 0, WAVE);
  q.next[base + lane] = q.buf[lane];
  q.cnt -= WAVE;
  const uint32_t rest = (uint32_t)lane < q.cnt ? q.buf[WAVE + lane] : 0u;
  wave_lds_sync();
  if ((uint32_t)lane < q.cnt) q.buf[lane] = rest;
  wave_lds_sync();
}

// the staged remainder (every lane calls, converged, before the wave exits)
__device__ inline void wq_flush(WaveQ &q) {
  if (!q.cnt) return;
  const int lane = lane_id();
  wave_lds_sync();
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(q.nnext, q.cnt);
  base = __shfl(base, 0, WAVE);
  if ((uint32_t)lane < q.cnt) q.next[base + lane] = q.buf[lane];
  q.cnt = 0;
}

// one arc step (every lane calls, converged): relax arc a with label L
__device__ inline void sssp_arc(const uint32_t *col, const uint32_t *w, uint64_t *labels, bool valid, uint64_t a,
                                uint64_t L, WaveQ &q, uint32_t *stamp, uint32_t iter) {
  bool add = false;
  uint32_t y = 0;
  if (valid) {
    y = col[a];
    const uint64_t nl = L + ((uint64_t)(w ? w[a] : 1u) << 32);
    if (nl < __hip_atomic_load(&labels[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      const uint64_t old = atomicMin((unsigned long long *)&labels[y], (unsigned long long)nl);
      if (nl < old) add = atomicMax(&stamp[y], iter) < iter;
    }
  }
  wq_push(q, add, y);
}

// One lane per frontier vertex: short rows flattened over the wave, long rows
// queued for k_sssp_heavy (one wave per row).
__global__ __launch_bounds__(256) void k_sssp_push(const uint64_t *row_ptr, const uint32_t *col,
                                                   const uint32_t *w, uint64_t *labels,
                                                   const uint32_t *front, const uint32_t *nfront,
                                                   uint32_t *next, uint32_t *nnext, uint32_t *stamp,
                                                   uint32_t iter, uint64_t *heavy, uint32_t *nheavy) {
  __shared__ uint32_t s_q[256 / WAVE][2 * WAVE];
  WaveQ q{s_q[threadIdx.x / WAVE], 0u, next, nnext};
  const uint32_t nf = *nfront;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x; b < nf; b += stride) {
    const uint64_t i = b + threadIdx.x;
    const bool want = i < nf;
    uint32_t v = 0;
    uint64_t a0 = 0, deg = 0, L = 0;
    if (want) {
      v = front[i];
      L = __hip_atomic_load(&labels[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      a0 = row_ptr[v];
      deg = row_ptr[v + 1] - a0;
    }
    const bool hv = want && deg > FLAT_MAX;
    push_pieces(heavy, nheavy + (iter & 1), hv, v, deg);
    flat_arcs(want && !hv, a0, deg, [&](bool valid, uint64_t a, int o) {
      sssp_arc(col, w, labels, valid, a, shfl_u64(L, o), q, stamp, iter);
    });
  }
  wq_flush(q);
}

// Long rows of iteration iter, one wave per row.  Also clears the count of
// the frontier iteration iter consumed (it receives the frontier after next)
// and the long-row counter of iteration iter + 1.
__global__ __launch_bounds__(256) void k_sssp_heavy(const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                                                    uint64_t *labels, uint32_t *next, uint32_t *nnext,
                                                    uint32_t *stamp, uint32_t iter, const uint64_t *heavy,
                                                    uint32_t *nheavy, uint32_t *nconsumed) {
  __shared__ uint32_t s_q[256 / WAVE][2 * WAVE];
  WaveQ q{s_q[threadIdx.x / WAVE], 0u, next, nnext};
  const int lane = lane_id();
  const uint32_t cnt = nheavy[iter & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *nconsumed = 0;
    nheavy[(iter + 1) & 1] = 0;
  }
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
  for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE; i < cnt; i += nw) {
    uint64_t a0, a1;
    const uint32_t v = piece_arcs(heavy[i], row_ptr, &a0, &a1);
    const uint64_t L = __hip_atomic_load(&labels[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint64_t c = a0; c < a1; c += WAVE)
      sssp_arc(col, w, labels, c + lane < a1, c + lane, L, q, stamp, iter);
  }
  wq_flush(q);
}

void sssp_alloc(Ctx &c, SsspWork &wk, uint32_t n, uint64_t m) {
  wk.front[0] = c.arena->get<uint32_t>(n + 1);
  wk.front[1] = c.arena->get<uint32_t>(n + 1);
  wk.flag = c.arena->get<uint32_t>(n);
  wk.heavy = c.arena->get<uint64_t>(piece_capacity(n, m));
  wk.ctr = c.arena->get<uint64_t>(4);
  fill_u32(c, wk.flag, n, 0);
  fill_u64(c, wk.ctr, 4, 0);
}

// Runs to the fixed point.  Returns the number of iterations.  Stamps grow
// monotonically across the calls on one workspace.  Labels travel against
// the arcs (over the in-arcs), so each vertex ends with the best label of the
// seeds it can reach: distances from every vertex TO the seed set.

uint32_t sssp_run(Ctx &c, const Graph &g, uint64_t *labels, const uint32_t *seeds, uint32_t nseeds,
                  SsspWork &wk, uint64_t) {
  if (nseeds == 0) return 0;
  uint32_t *cnt = reinterpret_cast<uint32_t *>(wk.ctr);  // cnt[0], cnt[1]: frontier sizes
  FL_HIP(hipMemcpyAsync(wk.front[0], seeds, (size_t)nseeds * 4, hipMemcpyDeviceToDevice, c.s));
  fill_u32(c, cnt, 4, 0);
  fill_u32(c, &cnt[0], 1, nseeds);
  uint32_t iters = 0, cur = 0;
  uint32_t nf = nseeds;
  while (nf) {
    // The kernel reads the frontier size on the device, so small frontiers
    // run several iterations per host check (an empty frontier costs one
    // short launch); large ones are checked after every iteration.
    // A frontier can grow by orders of magnitude within a burst: burst
    // launches get a grid for any frontier (blocks past the count exit).
    const uint32_t burst = nf > 65536 ? 1u : 8u;
    uint64_t blocks = ceil_div((uint64_t)nf, 256);
    if (burst > 1) blocks = std::max<uint64_t>(blocks, std::min<uint64_t>(ceil_div(g.n, 256), 2048));
    if (blocks > 16384) blocks = 16384;
    for (uint32_t b = 0; b < burst; ++b) {
      // cnt[cur ^ 1] (the next frontier's count) is zero: cleared at the
      // start or by the previous iteration's k_sssp_heavy
      const uint32_t stamp = ++wk.stamp;
      k_sssp_push<<<(uint32_t)blocks, 256, 0, c.s>>>(g.in_ptr, g.in_col, g.in_w, labels, wk.front[cur], &cnt[cur],
                                                      wk.front[cur ^ 1], &cnt[cur ^ 1], wk.flag, stamp,
                                                      wk.heavy, &cnt[2]);
      FL_LAUNCH_CHECK();
      k_sssp_heavy<<<HEAVY_BLOCKS, 256, 0, c.s>>>(g.in_ptr, g.in_col, g.in_w, labels, wk.front[cur ^ 1], &cnt[cur ^ 1],
                                         wk.flag, stamp, wk.heavy, &cnt[2], &cnt[cur]);
      FL_LAUNCH_CHECK();
      cur ^= 1;
      ++iters;
    }
    FL_HIP(hipMemcpyAsync(c.h_status, &cnt[cur], 4, hipMemcpyDeviceToHost, c.s));
    c.sync();
    nf = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
  }
  return iters;
}

}  // namespace fl
