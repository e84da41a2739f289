// fl_api.hip -- the C ABI (include/fl.h): parameter checks, workspace
// management and the solve driver that chains the phases
//   validate -> ranks/sketches -> gamma and ladder -> opening loop -> MIS ->
//   assignment -> objective.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "fl_ads.h"
#include "fl_common.h"
#include "fl_mis.h"
#include "fl_open.h"

namespace fl {

static std::atomic<int> g_last_hip{0};
void set_last_hip_error(int e) { g_last_hip.store(e); }

// ---- device memory: hipMalloc/hipFree, or the caller's hooks --------------
struct AllocHooks {
  fl_alloc_fn alloc = nullptr;
  fl_free_fn free_fn = nullptr;
  void *ctx = nullptr;
};
struct HookedBlock {
  AllocHooks h;
  size_t bytes;
  int device;
};
static std::mutex g_hooks_mu;
static AllocHooks g_hooks;
static std::unordered_map<void *, HookedBlock> g_hooked;  // blocks from the hooks, by address
static std::atomic<int> g_servers{0};

// nullptr on failure
static void *dev_alloc(size_t bytes) {
  AllocHooks h;
  {
    std::lock_guard<std::mutex> lk(g_hooks_mu);
    h = g_hooks;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (h.alloc) {
    void *p = h.alloc(bytes, dev, h.ctx);
    if (p) {
      std::lock_guard<std::mutex> lk(g_hooks_mu);
      g_hooked[p] = HookedBlock{h, bytes, dev};
    }
    return p;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}
// frees through whatever allocated the block
static void dev_free(void *p) {
  if (!p) return;
  HookedBlock b;
  bool hooked = false;
  {
    std::lock_guard<std::mutex> lk(g_hooks_mu);
    auto it = g_hooked.find(p);
    if (it != g_hooked.end()) {
      b = it->second;
      g_hooked.erase(it);
      hooked = true;
    }
  }
  if (hooked) b.h.free_fn(p, b.bytes, b.device, b.h.ctx);
  else (void)hipFree(p);
}

void Arena::reserve(size_t bytes) {
  if (fixed_) return;  // a fixed buffer never grows; get() reports exhaustion
  bytes = (bytes + (size_t(1) << 21) - 1) & ~((size_t(1) << 21) - 1);
  if (bytes <= cap_) return;
  release();
  void *p = dev_alloc(bytes);
  if (std::getenv("FL_DEBUG")) std::fprintf(stderr, "[fl] workspace %zu bytes: %s\n", bytes, p ? "ok" : "failed");
  if (!p) throw Error{FL_ENOMEM};
  base_ = static_cast<char *>(p);
  cap_ = bytes;
  used_ = 0;
}
void Arena::release() {
  if (!fixed_) dev_free(base_);
  fixed_ = false;
  base_ = nullptr;
  cap_ = used_ = 0;
}

struct DeviceCache {
  std::mutex mu;
  Arena arena;
  uint64_t *h_status = nullptr;
  bool timing = true;  // per-phase HIP events
  void release_all() {
    arena.release();
    if (h_status) (void)hipHostFree(h_status);
    h_status = nullptr;
  }
};
static DeviceCache g_cache[64];

// Workers of fl_solve_batch: a group is split into up to BATCH_WORKERS
// sub-unions solved at once on their own streams, so that one sub-union's
// host synchronisations and small launches overlap another's kernels.
constexpr int BATCH_WORKERS = 3;
struct BatchPool {
  DeviceCache dc[BATCH_WORKERS];
  hipStream_t st[BATCH_WORKERS] = {};
};
static BatchPool g_pool[64];

// Workspace of fl_solve_static: one fixed device array, never allocated or
// freed by the library.  Each device that loads the library holds its own
// copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// name denotes a host-side stand-in, not device memory).
static __device__ __align__(256) char scratch[FL_STATIC_SCRATCH_BYTES];
struct StaticWorkspace {
  std::mutex mu;
  char *ptr = nullptr;      // device address of `scratch` on this device
  DeviceCache dc;           // arena over ptr, host status words below, no timing events
  uint64_t h_status[4096];  // readback words (ordinary host memory, no pinned allocation)
};
static StaticWorkspace g_static[64];

static DeviceCache &cache_for_current() {
  int dev = 0;
  FL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error{FL_EINVAL};
  return g_cache[dev];
}

static void ensure_host_status(DeviceCache &dc) {
  if (!dc.h_status) FL_HIP(hipHostMalloc((void **)&dc.h_status, 4096 * 8, hipHostMallocDefault));
}

// ---------------------------------------------------------------------------
// small kernels of the driver
// ---------------------------------------------------------------------------
__global__ void k_fac_flags(uint32_t n, const uint32_t *fac_cost, uint32_t *flag) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = fac_cost[v] != FL_NOT_FACILITY ? 1u : 0u;
}
__global__ void k_fac_index(uint32_t n, const uint32_t *flag, const uint64_t *pos, uint32_t *fac_list,
                            uint32_t *fac_idx) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (flag[v]) {
    fac_list[pos[v]] = (uint32_t)v;
    fac_idx[v] = (uint32_t)pos[v];
  } else {
    fac_idx[v] = INF32;
  }
}
// gamma labels: facility f starts at (c(f) << 32 | f)
__global__ void k_gamma_init(uint32_t n, const uint32_t *fac_cost, uint64_t *lab) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    const uint32_t c = fac_cost[v];
    lab[v] = c != FL_NOT_FACILITY ? (((uint64_t)c << 32) | v) : INF64;
  }
}
// served clients, gamma, counts per graph: fields nC, nCeff, nUF0, max gamma
enum { CL_NC = 0, CL_NCEFF, CL_NUF0, CL_GMAX, CL_NFIELD };
__global__ void k_clients(uint32_t n, const uint32_t *gid, const uint8_t *is_client, const uint64_t *gl,
                          const uint32_t *fac_cost, uint8_t *ceff, uint64_t *ctr, uint32_t stripes) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < n;
  bool cl = false, ce = false, uf = false;
  uint64_t gmax = 0;
  uint32_t g = 0;
  if (valid) {
    g = seg_of(gid, (uint32_t)v);
    cl = is_client ? is_client[v] != 0 : true;
    ce = cl && gl[v] != INF64;
    uf = ce && fac_cost[v] != FL_NOT_FACILITY;
    ceff[v] = ce ? 1 : 0;
    if (ce) gmax = gl[v] >> 32;
  }
  unsigned long long *c = (unsigned long long *)ctr;
  seg_add(c, valid, g, CL_NC, CL_NFIELD, stripes, cl ? 1 : 0);
  seg_add(c, valid, g, CL_NCEFF, CL_NFIELD, stripes, ce ? 1 : 0);
  seg_add(c, valid, g, CL_NUF0, CL_NFIELD, stripes, uf ? 1 : 0);
  seg_max(c, valid, g, CL_GMAX, CL_NFIELD, stripes, gmax);
}
__global__ void k_scatter_q(uint32_t nF, const uint32_t *fac_list, const double *qf, double *q) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nF) q[fac_list[i]] = qf[i];
}
__global__ void k_assign_init(uint32_t n, const uint8_t *open, uint64_t *lab, uint32_t *flag) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    lab[v] = open[v] ? (uint64_t)v : INF64;
    flag[v] = open[v] ? 1u : 0u;
  }
}
__global__ void k_compact_u32(uint32_t n, const uint32_t *flag, const uint64_t *pos, uint32_t *out) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && flag[v]) out[pos[v]] = (uint32_t)v;
}
// Reach guard (directed graphs; never fires on an undirected one): a served
// client that reaches no facility of S opens its gamma minimiser (low half of
// its gamma label), which it reaches by definition.  Such a facility was
// closed (it would be in reach otherwise): it is marked 2 and counted once
// by the kernel below, which writes it back as 1.
__global__ void k_reach_guard(uint32_t n, const uint8_t *ceff, const uint64_t *lab, const uint64_t *gam_lab,
                              uint8_t *open, uint32_t *cnt) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && ceff[v] && lab[v] == INF64) {
    open[(uint32_t)(gam_lab[v] & 0xFFFFFFFFu)] = 2;
    atomicAdd(cnt, 1u);
  }
}
// assignment outputs (facility ids local to the graph) and the objective per
// graph: fields cost, n_open, n_guard, n_reach_guard
enum { AO_COST = 0, AO_NOPEN, AO_NGUARD, AO_NREACH, AO_NFIELD };
__global__ void k_assign_out(uint32_t n, const uint32_t *gid, const SegInfo *seg, const uint8_t *ceff,
                             const uint64_t *lab, uint8_t *open, const uint32_t *fac_cost,
                             const uint32_t *orung, uint32_t *assign, uint32_t *dist, uint64_t *ctr,
                             uint32_t stripes) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = v < n;
  uint64_t cost = 0, no = 0, ng = 0, nr = 0;
  uint32_t g = 0;
  if (valid) {
    g = seg_of(gid, (uint32_t)v);
    if (ceff[v]) {
      const uint64_t L = lab[v];
      assign[v] = (uint32_t)(L & 0xFFFFFFFFu) - seg[g].base;
      const uint32_t d = (uint32_t)(L >> 32);
      if (dist) dist[v] = d;
      cost += d;
    } else {
      assign[v] = FL_NONE;
      if (dist) dist[v] = FL_NONE;
    }
    if (open[v]) {
      cost += fac_cost[v];
      no = 1;
      if (open[v] == 2) {
        nr = 1;
        open[v] = 1;
      }
    }
    if (orung[v] == FL_RUNG_GUARD) ng = 1;
  }
  unsigned long long *c = (unsigned long long *)ctr;
  seg_add(c, valid, g, AO_COST, AO_NFIELD, stripes, cost);
  seg_add(c, valid, g, AO_NOPEN, AO_NFIELD, stripes, no);
  seg_add(c, valid, g, AO_NGUARD, AO_NFIELD, stripes, ng);
  seg_add(c, valid, g, AO_NREACH, AO_NFIELD, stripes, nr);
}

// ---- union of several graphs ------------------------------------------------
struct UnionDesc {
  const uint64_t *row_ptr;
  const uint32_t *col, *w, *fac_cost;
  const uint8_t *is_client;
  uint32_t n, base;
  uint64_t m, abase;
};
// vertex arrays of the union; grid (x: vertex blocks, y: graph)
__global__ void k_union_vertices(const UnionDesc *d, uint32_t *gid, uint64_t *row_ptr, uint32_t *fac_cost,
                                 uint8_t *is_client) {
  const uint32_t g = blockIdx.y;
  const UnionDesc D = d[g];
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < D.n; v += gridDim.x * blockDim.x) {
    const uint32_t u = D.base + v;
    gid[u] = g;
    row_ptr[u] = D.abase + D.row_ptr[v];
    fac_cost[u] = D.fac_cost[v];
    is_client[u] = D.is_client ? (D.is_client[v] != 0) : 1;
  }
}
// arcs of the union (ids shifted by the graph's base; unit graphs get w = 1)
__global__ void k_union_arcs(const UnionDesc *d, uint32_t *col, uint32_t *w) {
  const uint32_t g = blockIdx.y;
  const UnionDesc D = d[g];
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < D.m;
       a += (uint64_t)gridDim.x * blockDim.x) {
    col[D.abase + a] = D.col[a] + D.base;
    if (w) w[D.abase + a] = D.w ? D.w[a] : 1u;
  }
}
// per-graph caller outputs from the union arrays; grid (x: vertex blocks, y: graph)
struct OutDesc {
  uint8_t *open;
  uint32_t *assign, *dist, *open_rung, *freeze_rung;
  double *q;
  uint32_t n, base;
};
__global__ void k_scatter_out(const OutDesc *d, const uint8_t *open, const uint32_t *assign, const uint32_t *dist,
                              const uint32_t *orung, const uint32_t *frz, const double *q) {
  const OutDesc D = d[blockIdx.y];
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < D.n; v += gridDim.x * blockDim.x) {
    const uint32_t u = D.base + v;
    D.open[v] = open[u];
    D.assign[v] = assign[u];
    if (D.dist) D.dist[v] = dist[u];
    if (D.open_rung) D.open_rung[v] = orung[u];
    if (D.freeze_rung) D.freeze_rung[v] = frz[u];
    if (D.q) D.q[v] = q[u];
  }
}
// pos[] at each graph's first vertex and at the end: facility counts per graph
__global__ void k_pick_u64(const uint64_t *src, const uint32_t *idx, uint32_t cnt, uint64_t *dst) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) dst[i] = src[idx[i]];
}
// largest arc weight of each graph of a batch; grid (x: arc blocks, y: graph)
struct WeightDesc {
  const uint32_t *w;
  uint64_t m;
};
__global__ __launch_bounds__(256) void k_max_weights(const WeightDesc *d, uint32_t *out) {
  const WeightDesc D = d[blockIdx.y];
  uint32_t mx = 0;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < D.m; a += (uint64_t)gridDim.x * blockDim.x)
    mx = D.w[a] > mx ? D.w[a] : mx;
  for (int o = WAVE / 2; o >= 1; o >>= 1) {
    const uint32_t t = __shfl_xor(mx, o, WAVE);
    mx = t > mx ? t : mx;
  }
  if (lane_id() == 0 && mx) atomicMax(&out[blockIdx.y], mx);
}

// Largest weight of each graph (1 for unit weights, at least 1), read before
// a batch is cut into groups: a group's slot rings hold max weight + 1
// distances, so its memory estimate needs the bound.  Nothing else is
// checked here; each group's solve validates its graphs, weights included.
static std::vector<uint32_t> batch_max_weights(Ctx &c, const fl_problem *const *ps, uint32_t G) {
  std::vector<uint32_t> mw(G, 1u);
  std::vector<WeightDesc> hd;
  std::vector<uint32_t> idx;
  uint64_t mmax = 0;
  for (uint32_t g = 0; g < G; ++g)
    if (ps[g]->w && ps[g]->n_arcs) {
      hd.push_back(WeightDesc{ps[g]->w, ps[g]->n_arcs});
      idx.push_back(g);
      mmax = std::max<uint64_t>(mmax, ps[g]->n_arcs);
    }
  if (hd.empty()) return mw;
  const uint32_t W = (uint32_t)hd.size();
  WeightDesc *dd = c.arena->get<WeightDesc>(W);
  uint32_t *dout = c.arena->get<uint32_t>(W);
  FL_HIP(hipMemcpyAsync(dd, hd.data(), W * sizeof(WeightDesc), hipMemcpyHostToDevice, c.s));
  fill_u32(c, dout, W, 0);
  const uint32_t bx = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(ceil_div(mmax, 256 * 64), 1), 64);
  for (uint32_t g0 = 0; g0 < W; g0 += 65535) {
    const uint32_t gy = std::min<uint32_t>(W - g0, 65535);
    k_max_weights<<<dim3(bx, gy), 256, 0, c.s>>>(dd + g0, dout + g0);
    FL_LAUNCH_CHECK();
  }
  std::vector<uint32_t> h(W);
  FL_HIP(hipMemcpyAsync(h.data(), dout, W * 4, hipMemcpyDeviceToHost, c.s));
  c.sync();
  for (uint32_t i = 0; i < W; ++i) mw[idx[i]] = std::max(h[i], 1u);
  return mw;
}

static int check_params(const fl_problem *p, const fl_params *prm) {
  if (!p || !prm) return FL_EINVAL;
  if (p->n == 0 || p->n >= 0xFFFFFFFFu) return FL_EINVAL;
  if (!p->row_ptr || (p->n_arcs && !p->col)) return FL_EINVAL;
  if (prm->k == 0) return FL_EINVAL;
  if (!(prm->eps > 0.0) || !std::isfinite(prm->eps)) return FL_EINVAL;
  if (prm->k > MAX_K) return FL_ENOTIMPL;
  return FL_OK;
}

static size_t estimate_bytes(uint32_t n, uint64_t m, uint64_t nF, uint32_t k, uint32_t cap, uint32_t NS) {
  size_t b = 0;
  b += (size_t)n * cap * 8;                // sketch ranks + distances
  b += (size_t)nF * cap * 4;               // HIP thresholds
  b += (size_t)n * 32;                     // outputs kept while the sketches are built
  const size_t ads = ads_scratch_bytes(n, m, k, NS);
  const size_t later = (size_t)NS * n * 8 + (size_t)NS * CNT_PAD * 4 + (size_t)n * 200 + (size_t)m / 64 +
                       (size_t)nF * 96;  // opening loop, MIS, assignment
  b += ads > later ? ads : later;
  b += (size_t)64 << 20;                   // counters, scans
  return b;
}
// extra bytes of a union of several graphs: CSR copy, graph ids, inputs and outputs
static size_t union_bytes(uint32_t G, uint64_t n, uint64_t m, bool weighted) {
  if (G <= 1) return 0;
  return (size_t)(n + 1) * 8 + (size_t)m * (weighted ? 8 : 4) + (size_t)n * (4 + 4 + 1) +
         (size_t)n * (1 + 4 + 4 + 4 + 4 + 8) + (size_t)G * 256 + ((size_t)4 << 20);
}

static double ms_between(hipEvent_t a, hipEvent_t b) {
  if (!a || !b) return 0.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

// One group of graphs with equal k, eps and flags (already checked by the
// caller), solved together as a disjoint union: every phase runs once for the
// whole group.  rc[i] receives each graph's code.
static void solve_group(const fl_problem *const *ps, const fl_params *const *pr, fl_result *const *outs,
                        uint32_t G0, hipStream_t s, DeviceCache &dc, std::vector<int> &rc_out, int depth = 0) {
  rc_out.assign(G0, FL_OK);
  ensure_host_status(dc);
  const uint32_t k = pr[0]->k;
  const double eps = pr[0]->eps;
  const uint32_t flags = pr[0]->flags;
  const bool directed = (flags & FL_FLAG_DIRECTED) != 0;
  uint64_t N0 = 0, M0 = 0;
  uint32_t nmax0 = 1;
  bool weighted0 = false;
  for (uint32_t i = 0; i < G0; ++i) {
    N0 += ps[i]->n;
    M0 += ps[i]->n_arcs;
    nmax0 = std::max(nmax0, ps[i]->n);
    weighted0 |= ps[i]->w != nullptr;
  }
  if (N0 >= 0xFFFFFFFFull) {
    for (auto &r : rc_out) r = FL_ENOMEM;
    return;
  }
  const uint32_t cap0 = ads_capacity(nmax0, k);
  const size_t tr0 = directed ? transpose_bytes((uint32_t)N0, M0, weighted0) : 0;
  dc.arena.reserve(estimate_bytes((uint32_t)N0, M0, N0, k, cap0, 2) + union_bytes(G0, N0, M0, weighted0) + tr0);
  dc.arena.reset();
  Ctx c;
  c.s = s;
  c.arena = &dc.arena;
  c.h_status = dc.h_status;
  c.timing = dc.timing;

  hipEvent_t ev[8] = {};
  if (c.timing)
    for (auto &e : ev) FL_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 8; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};
  auto mark = [&](int i) {
    if (ev[i]) FL_HIP(hipEventRecord(ev[i], s));
  };
  mark(0);

  // ---- validation per graph; failing graphs leave the group
  std::vector<uint32_t> mw(G0, 1), mc(G0, 0);
  if (G0 == 1) {
    rc_out[0] = validate_graph(c, ps[0], directed, &mw[0], &mc[0]);
  } else {
    validate_graphs(c, ps, G0, directed, rc_out, mw, mc);
  }
  std::vector<uint32_t> act;  // indices of the graphs that go on
  for (uint32_t i = 0; i < G0; ++i) {
    if (rc_out[i]) continue;
    const fl_problem *p = ps[i];
    const uint64_t bound = (uint64_t)(p->n - 1) * (p->w ? mw[i] : 1u) + mc[i];
    if (bound >= 0xFFFFFFFFull) rc_out[i] = FL_ERANGE;
    else if (p->w && mw[i] > MAX_W) rc_out[i] = FL_ENOTIMPL;
    else act.push_back(i);
  }
  if (act.empty()) return;
  if (act.size() < G0) {
    // solve the valid ones alone: the union must hold valid graphs only
    std::vector<const fl_problem *> ps2;
    std::vector<const fl_params *> pr2;
    std::vector<fl_result *> out2;
    for (uint32_t i : act) {
      ps2.push_back(ps[i]);
      pr2.push_back(pr[i]);
      out2.push_back(outs[i]);
    }
    std::vector<int> rc2;
    solve_group(ps2.data(), pr2.data(), out2.data(), (uint32_t)act.size(), s, dc, rc2, depth);
    for (size_t j = 0; j < act.size(); ++j) rc_out[act[j]] = rc2[j];
    return;
  }
  const uint32_t G = G0;
  const uint32_t n = (uint32_t)N0;
  uint32_t max_w = 1;
  for (uint32_t i = 0; i < G; ++i)
    if (ps[i]->w) max_w = std::max(max_w, mw[i]);
  const bool weighted = weighted0;
  const uint32_t NS = (weighted ? max_w : 1u) + 1;
  const size_t need = estimate_bytes(n, M0, n, k, cap0, NS) + union_bytes(G, N0, M0, weighted) + tr0;
  if (!dc.arena.fixed() && need > dc.arena.capacity()) {
    if (depth > 0) {
      for (auto &r : rc_out) r = FL_ENOMEM;
      return;
    }
    dc.arena.reserve(need);
    return solve_group(ps, pr, outs, G0, s, dc, rc_out, depth + 1);  // restart with the larger arena
  }

  // ---- the union (one graph: the caller's arrays as they are)
  std::vector<uint32_t> hbase(G);
  {
    uint64_t b = 0;
    for (uint32_t i = 0; i < G; ++i) {
      hbase[i] = (uint32_t)b;
      b += ps[i]->n;
    }
  }
  std::vector<SegInfo> hseg(G);
  for (uint32_t i = 0; i < G; ++i) hseg[i] = seg_info(hbase[i], ps[i]->n, pr[i]->seed);
  SegInfo *seg = c.arena->get<SegInfo>(G);
  FL_HIP(hipMemcpyAsync(seg, hseg.data(), G * sizeof(SegInfo), hipMemcpyHostToDevice, s));
  const uint32_t *gid = nullptr;
  const uint32_t *fac_cost = ps[0]->fac_cost;
  const uint8_t *is_client = ps[0]->is_client;
  Graph g{n, M0, ps[0]->row_ptr, ps[0]->col, ps[0]->w, weighted ? max_w : 1u};
  if (G > 1) {
    std::vector<UnionDesc> hd(G);
    uint64_t ab = 0;
    uint32_t mx_blocks = 1;
    uint64_t mx_m = 1;
    for (uint32_t i = 0; i < G; ++i) {
      const fl_problem *p = ps[i];
      hd[i] = UnionDesc{p->row_ptr, p->col, p->w, p->fac_cost, p->is_client, p->n, hbase[i], p->n_arcs, ab};
      ab += p->n_arcs;
      mx_blocks = std::max<uint32_t>(mx_blocks, (uint32_t)ceil_div(p->n, 256));
      mx_m = std::max<uint64_t>(mx_m, p->n_arcs);
    }
    UnionDesc *dd = c.arena->get<UnionDesc>(G);
    FL_HIP(hipMemcpyAsync(dd, hd.data(), G * sizeof(UnionDesc), hipMemcpyHostToDevice, s));
    uint32_t *d_gid = c.arena->get<uint32_t>(n);
    uint64_t *d_rp = c.arena->get<uint64_t>((size_t)n + 1);
    uint32_t *d_col = c.arena->get<uint32_t>(M0 ? M0 : 1);
    uint32_t *d_w = weighted ? c.arena->get<uint32_t>(M0 ? M0 : 1) : nullptr;
    uint32_t *d_fc = c.arena->get<uint32_t>(n);
    uint8_t *d_cl = c.arena->get<uint8_t>(n);
    const uint32_t vbx = std::min<uint32_t>(mx_blocks, 1024);
    k_union_vertices<<<dim3(vbx, G), 256, 0, s>>>(dd, d_gid, d_rp, d_fc, d_cl);
    FL_LAUNCH_CHECK();
    fill_u64(c, d_rp + n, 1, M0);
    const uint32_t abx = (uint32_t)std::min<uint64_t>(ceil_div(mx_m, 256 * 8), 1024);
    k_union_arcs<<<dim3(abx, G), 256, 0, s>>>(dd, d_col, d_w);
    FL_LAUNCH_CHECK();
    c.sync();  // hd is read by the copy above
    gid = d_gid;
    fac_cost = d_fc;
    is_client = d_cl;
    g = Graph{n, M0, d_rp, d_col, d_w, weighted ? max_w : 1u};
  }
  set_in_arcs(c, g, directed);
  mark(1);

  // ---- facilities
  uint32_t *flag = c.arena->get<uint32_t>(n);
  uint64_t *pos = c.arena->get<uint64_t>((size_t)n + 1);
  uint32_t *fac_list = c.arena->get<uint32_t>(n);
  uint32_t *fac_idx = c.arena->get<uint32_t>(n);
  const uint32_t vb = (uint32_t)ceil_div(n, 256);
  k_fac_flags<<<vb, 256, 0, s>>>(n, fac_cost, flag);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, flag, pos, n);
  k_fac_index<<<vb, 256, 0, s>>>(n, flag, pos, fac_list, fac_idx);
  FL_LAUNCH_CHECK();
  std::vector<uint64_t> nF_g(G);
  uint32_t nF = 0;
  {
    std::vector<uint32_t> hidx(G + 1);
    for (uint32_t i = 0; i < G; ++i) hidx[i] = hbase[i];
    hidx[G] = n;
    uint32_t *didx = c.arena->get<uint32_t>(G + 1);
    uint64_t *dval = c.arena->get<uint64_t>(G + 1);
    FL_HIP(hipMemcpyAsync(didx, hidx.data(), (G + 1) * 4, hipMemcpyHostToDevice, s));
    k_pick_u64<<<(uint32_t)ceil_div(G + 1, 256), 256, 0, s>>>(pos, didx, G + 1, dval);
    FL_LAUNCH_CHECK();
    std::vector<uint64_t> hv(G + 1);
    FL_HIP(hipMemcpyAsync(hv.data(), dval, (G + 1) * 8, hipMemcpyDeviceToHost, s));
    c.sync();
    for (uint32_t i = 0; i < G; ++i) nF_g[i] = hv[i + 1] - hv[i];
    nF = (uint32_t)hv[G];
  }

  // ---- sketches (Sec. 3.3)
  AdsConfig acfg{k, gid, seg, flags, nF, fac_idx, fac_list, nmax0};
  AdsOut ads;
  int rc = ads_build(c, g, acfg, ads);
  if (rc) {
    for (auto &r : rc_out) r = rc;
    return;
  }
  std::vector<uint64_t> relax, entries;
  ads_totals(c, g, gid, G, ads.cnt, relax, entries);
  mark(2);

  // ---- gamma (Sec. 4.1) and served clients
  const uint32_t stripes = G == 1 ? 64 : 1;
  uint64_t *gl = c.arena->get<uint64_t>(n);
  uint8_t *ceff = c.arena->get<uint8_t>(n);
  uint64_t *ctr = c.arena->get<uint64_t>((size_t)G * 4 * stripes);
  k_gamma_init<<<vb, 256, 0, s>>>(n, fac_cost, gl);
  FL_LAUNCH_CHECK();
  SsspWork wk;
  sssp_alloc(c, wk, n, g.m);
  sssp_run(c, g, gl, fac_list, nF, wk, 0);
  fill_u64(c, ctr, (size_t)G * CL_NFIELD * stripes, 0);
  k_clients<<<vb, 256, 0, s>>>(n, gid, is_client, gl, fac_cost, ceff, ctr, stripes);
  FL_LAUNCH_CHECK();
  const std::vector<uint64_t> cs = read_seg_ctr(c, ctr, G, CL_NFIELD, stripes, true);
  const double one_eps = 1.0 + eps;
  std::vector<std::vector<double>> lad(G);
  OpenIn oi{&g, G, gid, seg, nF, fac_list, fac_idx, fac_cost, &ads, ceff, nF_g, {}, {}, gl, eps, &lad};
  oi.nCeff.resize(G);
  oi.nUF0.resize(G);
  for (uint32_t i = 0; i < G; ++i) {
    const uint64_t nC = cs[i * CL_NFIELD + CL_NC], nCeff = cs[i * CL_NFIELD + CL_NCEFF];
    const uint64_t gamma = cs[i * CL_NFIELD + CL_GMAX];
    oi.nCeff[i] = nCeff;
    oi.nUF0[i] = cs[i * CL_NFIELD + CL_NUF0];
    outs[i]->stats.gamma = gamma;
    outs[i]->n_unreachable = (uint32_t)(nC - nCeff);
    lad[i].assign(1, 0.0);
    if (nF_g[i] > 0 && nCeff > 0) {
      const double Mq = (double)(nF_g[i] * nCeff);
      lad[i][0] = ((double)gamma / (Mq * Mq)) * one_eps;
    }
    lad[i].push_back(lad[i][0] * one_eps);
    outs[i]->stats.alpha0 = lad[i][0];
  }
  mark(3);

  // ---- outputs: the caller's arrays for one graph, union arrays otherwise
  fl_result *o0 = outs[0];
  uint8_t *open_u = G == 1 ? o0->open : c.arena->get<uint8_t>(n);
  uint32_t *assign_u = G == 1 ? o0->assign : c.arena->get<uint32_t>(n);
  uint32_t *dist_u = G == 1 ? o0->dist : c.arena->get<uint32_t>(n);
  uint32_t *orung = (G == 1 && o0->open_rung) ? o0->open_rung : c.arena->get<uint32_t>(n);
  uint32_t *frz = (G == 1 && o0->freeze_rung) ? o0->freeze_rung : c.arena->get<uint32_t>(n);
  bool want_q = false;
  for (uint32_t i = 0; i < G; ++i) want_q |= outs[i]->q != nullptr;
  double *q_u = nullptr;
  if (want_q) q_u = G == 1 ? o0->q : c.arena->get<double>(n);

  // ---- opening loop (Alg. 4, Alg. 5)
  double *qf = c.arena->get<double>(nF ? nF : 1);
  OpenOut oo{orung, frz, qf, {}, {}, {}};
  rc = open_phase(c, oi, oo);
  if (rc) {
    for (auto &r : rc_out) r = rc;
    return;
  }
  if (q_u) {
    fill_f64(c, q_u, n, 0.0);
    if (nF) {
      k_scatter_q<<<(uint32_t)ceil_div(nF, 256), 256, 0, s>>>(nF, fac_list, qf, q_u);
      FL_LAUNCH_CHECK();
    }
  }
  mark(4);

  // ---- MIS per rung (Sec. 4.3, Alg. 6)
  MisIn mi{&g, G, gid, seg, oo.rungs, &lad, eps, orung, frz, (flags & FL_FLAG_LUBY_MIS) != 0};
  std::vector<uint32_t> mis_rounds;
  rc = mis_phase(c, mi, open_u, mis_rounds);
  if (rc) {
    for (auto &r : rc_out) r = rc;
    return;
  }
  mark(5);

  // ---- assignment and objective (Sec. 3.1)
  uint64_t *al = c.arena->get<uint64_t>(n);
  uint32_t *slist = c.arena->get<uint32_t>(n);
  uint32_t *rgc = c.arena->get<uint32_t>(1);
  for (int pass = 0; pass < 2; ++pass) {
    k_assign_init<<<vb, 256, 0, s>>>(n, open_u, al, flag);
    FL_LAUNCH_CHECK();
    scan_u32_to_u64(c, flag, pos, n);
    k_compact_u32<<<vb, 256, 0, s>>>(n, flag, pos, slist);
    FL_LAUNCH_CHECK();
    FL_HIP(hipMemcpyAsync(c.h_status, pos + n, 8, hipMemcpyDeviceToHost, s));
    c.sync();
    const uint32_t nS = (uint32_t)c.h_status[0];
    sssp_run(c, g, al, slist, nS, wk, 0);
    if (!directed || pass == 1) break;
    fill_u32(c, rgc, 1, 0);
    k_reach_guard<<<vb, 256, 0, s>>>(n, ceff, al, gl, open_u, rgc);
    FL_LAUNCH_CHECK();
    FL_HIP(hipMemcpyAsync(c.h_status, rgc, 4, hipMemcpyDeviceToHost, s));
    c.sync();
    if ((c.h_status[0] & 0xFFFFFFFFu) == 0) break;  // every served client reaches S
  }
  uint64_t *actr = c.arena->get<uint64_t>((size_t)G * AO_NFIELD * stripes);
  fill_u64(c, actr, (size_t)G * AO_NFIELD * stripes, 0);
  k_assign_out<<<vb, 256, 0, s>>>(n, gid, seg, ceff, al, open_u, fac_cost, orung, assign_u, dist_u, actr,
                                  stripes);
  FL_LAUNCH_CHECK();
  if (G > 1) {
    std::vector<OutDesc> hd(G);
    uint32_t mx_blocks = 1;
    for (uint32_t i = 0; i < G; ++i) {
      fl_result *o = outs[i];
      hd[i] = OutDesc{o->open, o->assign, o->dist, o->open_rung, o->freeze_rung, o->q, ps[i]->n, hbase[i]};
      mx_blocks = std::max<uint32_t>(mx_blocks, (uint32_t)ceil_div(ps[i]->n, 256));
    }
    OutDesc *dd = c.arena->get<OutDesc>(G);
    FL_HIP(hipMemcpyAsync(dd, hd.data(), G * sizeof(OutDesc), hipMemcpyHostToDevice, s));
    k_scatter_out<<<dim3(std::min<uint32_t>(mx_blocks, 1024), G), 256, 0, s>>>(dd, open_u, assign_u, dist_u,
                                                                               orung, frz, q_u);
    FL_LAUNCH_CHECK();
    c.sync();  // hd is read by the copy above
  }
  const std::vector<uint64_t> ao = read_seg_ctr(c, actr, G, AO_NFIELD, stripes);
  mark(6);
  if (ev[6]) FL_HIP(hipEventSynchronize(ev[6]));
  else c.sync();
  for (uint32_t i = 0; i < G; ++i) {
    fl_result *o = outs[i];
    if (oo.rc[i] != FL_OK) {
      rc_out[i] = oo.rc[i];
      o->n_open = 0;
      continue;
    }
    o->total_cost = ao[i * AO_NFIELD + AO_COST];
    o->n_open = (uint32_t)ao[i * AO_NFIELD + AO_NOPEN];
    fl_stats &st = o->stats;
    st.n_guard = (uint32_t)ao[i * AO_NFIELD + AO_NGUARD];
    st.n_reach_guard = (uint32_t)ao[i * AO_NFIELD + AO_NREACH];
    st.relax_alg = relax[i];
    st.ads_entries = entries[i];
    st.rungs = oo.rungs[i];
    st.mis_rounds = mis_rounds[i];
    // group-wide figures: rounds, executed relaxations and times are those of
    // the whole union
    st.ads_rounds = ads.rounds;
    st.relax_exec = ads.relax_exec;
    st.ms_ads_kernel = ads.kernel_ms;
    st.ms_ads_merge = ads.merge_ms;
    st.ads_kernel_launches = ads.launches;
    st.ms_validate = ms_between(ev[0], ev[1]);
    st.ms_ads = ms_between(ev[1], ev[2]);
    st.ms_gamma = ms_between(ev[2], ev[3]);
    st.ms_open = ms_between(ev[3], ev[4]);
    st.ms_mis = ms_between(ev[4], ev[5]);
    st.ms_assign = ms_between(ev[5], ev[6]);
    st.ms_total = ms_between(ev[0], ev[6]);
    st.workspace_bytes = c.arena->used();
  }
}

// ---------------------------------------------------------------------------
// serving: continuous batching over worker slots
// ---------------------------------------------------------------------------
struct Request {
  const fl_problem *p;
  const fl_params *prm;
  fl_result *out;
  uint64_t ticket;
  size_t bytes;  // workspace of this request alone
  int status = FL_EBUSY;
  bool done = false;
};

struct Server;
struct Slot {
  Server *srv = nullptr;
  DeviceCache dc;
  hipStream_t stream = nullptr;
  size_t cap = 0;  // workspace bytes this slot holds
  bool busy = false;
  std::thread th;
};

struct Server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<Slot *> slots;
};

static size_t group_bytes(const std::vector<Request *> &b) {
  uint64_t N = 0, M = 0;
  uint32_t nmax = 1;
  bool wt = false;
  for (const Request *r : b) {
    N += r->p->n;
    M += r->p->n_arcs;
    nmax = std::max(nmax, r->p->n);
    wt |= r->p->w != nullptr;
  }
  const uint32_t k = b[0]->prm->k;
  const uint32_t N32 = (uint32_t)std::min<uint64_t>(N, 0xFFFFFFFEull);
  return estimate_bytes(N32, M, N, k, ads_capacity(nmax, k), wt ? MAX_W + 1 : 2) +
         union_bytes((uint32_t)b.size(), N, M, wt) +
         ((b[0]->prm->flags & FL_FLAG_DIRECTED) ? transpose_bytes(N32, M, wt) : 0);
}

static bool same_group(const Request *a, const Request *b) {
  return a->prm->k == b->prm->k && a->prm->eps == b->prm->eps && a->prm->flags == b->prm->flags;
}

static void slot_main(Slot *sl) {
  Server &S = *sl->srv;
  (void)hipSetDevice(S.device);
  for (;;) {
    std::vector<Request *> batch;
    size_t need = 0;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      for (;;) {
        if (S.queue.empty()) {
          if (S.stop) return;
          S.cv_work.wait(lk);
          continue;
        }
        // the oldest request, then later ones of the same group while the
        // budget allows.  Workspaces of running slots count against the
        // budget; idle slots give theirs up when the room is needed.
        Request *head = S.queue.front();
        batch.assign(1, head);
        need = group_bytes(batch);
        size_t running = 0;
        for (Slot *x : S.slots)
          if (x != sl && x->busy) running += x->cap;
        if (running + need > S.budget && running > 0) {
          S.cv_work.wait(lk);  // wait for a running slot to finish
          continue;
        }
        // share the waiting requests among the idle workers (this one included)
        size_t idle = 0;
        for (Slot *x : S.slots) idle += x->busy ? 0 : 1;
        const size_t take = std::max<size_t>(1, (S.queue.size() + idle - 1) / std::max<size_t>(idle, 1));
        for (size_t i = 1; i < S.queue.size() && batch.size() < std::min<size_t>(take, 4096); ++i) {
          Request *r = S.queue[i];
          if (!same_group(head, r)) continue;
          batch.push_back(r);
          const size_t nb = group_bytes(batch);
          if (running + nb > S.budget) {
            batch.pop_back();
            continue;
          }
          need = nb;
        }
        for (Request *r : batch)
          for (auto it = S.queue.begin(); it != S.queue.end(); ++it)
            if (*it == r) {
              S.queue.erase(it);
              break;
            }
        // make room: this slot's workspace grows to `need` (or is dropped
        // and rebuilt), idle slots release theirs while the total is over
        size_t total = running + std::max(need, sl->cap);
        for (Slot *x : S.slots) {
          if (total <= S.budget) break;
          if (x == sl || x->busy || x->cap == 0) continue;
          std::lock_guard<std::mutex> xl(x->dc.mu);
          x->dc.arena.release();
          total -= x->cap;
          x->cap = 0;
        }
        if (total > S.budget && sl->cap > need) {
          sl->dc.arena.release();
          sl->cap = 0;
        }
        sl->busy = true;
        sl->cap = std::max(need, sl->cap);
        break;
      }
    }
    std::vector<const fl_problem *> ps;
    std::vector<const fl_params *> pr;
    std::vector<fl_result *> os;
    for (Request *r : batch) {
      ps.push_back(r->p);
      pr.push_back(r->prm);
      os.push_back(r->out);
      r->out->n_open = 0;
      std::memset(&r->out->stats, 0, sizeof(r->out->stats));
    }
    std::vector<int> rc;
    try {
      std::lock_guard<std::mutex> lk(sl->dc.mu);
      sl->dc.arena.reserve(need);
      solve_group(ps.data(), pr.data(), os.data(), (uint32_t)batch.size(), sl->stream, sl->dc, rc);
    } catch (Error &e) {
      rc.assign(batch.size(), e.code);
    } catch (std::bad_alloc &) {
      rc.assign(batch.size(), FL_ENOMEM);
    }
    {
      std::lock_guard<std::mutex> lk(S.mu);
      // the workspace may have grown past the estimate
      sl->cap = sl->dc.arena.capacity();
      sl->busy = false;
      for (size_t i = 0; i < batch.size(); ++i) {
        Request *r = batch[i];
        r->status = rc[i];
        r->out->status = rc[i];
        if (rc[i] != FL_OK) r->out->n_open = 0;
        r->done = true;
      }
    }
    S.cv_done.notify_all();
    S.cv_work.notify_all();
  }
}

}  // namespace fl

struct fl_server {
  fl::Server s;
};

namespace fl {

// ---------------------------------------------------------------------------
// sketches for export
// ---------------------------------------------------------------------------
}  // namespace fl

struct fl_sketch {
  int device;
  uint32_t n, k;
  uint64_t total;
  uint64_t *off;
  uint32_t *rank, *dist, *thr;
  void *mem;
};

extern "C" {

int fl_solve(const fl_problem *p, const fl_params *prm, fl_result *out, void *stream) {
  if (out) out->n_open = 0;
  if (out) out->status = FL_EINVAL;
  try {
    if (out) std::memset(&out->stats, 0, sizeof(out->stats));
    int pc = fl::check_params(p, prm);
    if (pc) return pc;
    if (!p->fac_cost || !out || !out->open || !out->assign) return FL_EINVAL;
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    std::vector<int> rc;
    fl::solve_group(&p, &prm, &out, 1, (hipStream_t)stream, dc, rc);
    if (rc[0] != FL_OK) out->n_open = 0;
    out->status = rc[0];
    return rc[0];
  } catch (fl::Error &e) {
    if (out) out->n_open = 0;
    if (out) out->status = e.code;
    return e.code;
  } catch (std::bad_alloc &) {
    if (out) out->n_open = 0;
    if (out) out->status = FL_ENOMEM;
    return FL_ENOMEM;
  }
}

int fl_solve_static(const fl_problem *p, const fl_params *prm, fl_result *out, void *stream) {
  if (out) out->n_open = 0;
  if (out) out->status = FL_EINVAL;
  try {
    if (out) std::memset(&out->stats, 0, sizeof(out->stats));
    int pc = fl::check_params(p, prm);
    if (pc) return pc;
    if (!p->fac_cost || !out || !out->open || !out->assign) return FL_EINVAL;
    // the sketch rows alone must fit: refuse before any device work
    if ((uint64_t)p->n * fl::ads_capacity(p->n, prm->k) * 8ull > FL_STATIC_SCRATCH_BYTES) {
      out->status = FL_ENOMEM;
      return FL_ENOMEM;
    }
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return FL_EINVAL;
    fl::StaticWorkspace &w = fl::g_static[dev];
    std::lock_guard<std::mutex> lk(w.mu);
    if (!w.ptr) {
      // once per device, with that device current
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(fl::scratch));
      if (e != hipSuccess || !ptr) {
        fl::set_last_hip_error((int)e);
        out->status = FL_EHIP;
        return FL_EHIP;
      }
      w.ptr = static_cast<char *>(ptr);
      w.dc.arena.attach(w.ptr, FL_STATIC_SCRATCH_BYTES);
      w.dc.h_status = w.h_status;
      w.dc.timing = false;
    }
    w.dc.arena.reset();
    std::vector<int> rc(1, FL_OK);
    try {
      fl::solve_group(&p, &prm, &out, 1, (hipStream_t)stream, w.dc, rc);
    } catch (fl::Error &e) {
      rc[0] = e.code;
    } catch (std::bad_alloc &) {
      rc[0] = FL_ENOMEM;
    }
    if (rc[0] != FL_OK) {
      // work enqueued before the failure may still read the array: it must
      // end before the next call may use it
      (void)hipStreamSynchronize((hipStream_t)stream);
      out->n_open = 0;
    }
    out->status = rc[0];
    return rc[0];
  } catch (fl::Error &e) {
    if (out) out->n_open = 0;
    if (out) out->status = e.code;
    return e.code;
  } catch (std::bad_alloc &) {
    if (out) out->n_open = 0;
    if (out) out->status = FL_ENOMEM;
    return FL_ENOMEM;
  }
}

int fl_solve_batch(const fl_problem *ps, const fl_params *prms, fl_result *outs, uint32_t count,
                   void *stream) {
  if (count && (!ps || !prms || !outs)) return FL_EINVAL;
  try {
    std::vector<int> rc(count, FL_OK);
    std::vector<uint32_t> ok;
    for (uint32_t i = 0; i < count; ++i) {
      outs[i].n_open = 0;
      outs[i].status = FL_EINVAL;
      std::memset(&outs[i].stats, 0, sizeof(outs[i].stats));
      int pc = fl::check_params(&ps[i], &prms[i]);
      if (!pc && (!ps[i].fac_cost || !outs[i].open || !outs[i].assign)) pc = FL_EINVAL;
      rc[i] = pc;
      if (!pc) ok.push_back(i);
    }
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    // groups: equal (k, eps, flags); largest graphs first; each group within
    // a byte budget (sketch rows are sized by the group's largest graph)
    std::sort(ok.begin(), ok.end(), [&](uint32_t a, uint32_t b) {
      const fl_params &x = prms[a], &y = prms[b];
      if (x.k != y.k) return x.k < y.k;
      if (x.eps != y.eps) return x.eps < y.eps;
      if (x.flags != y.flags) return x.flags < y.flags;
      if (ps[a].n != ps[b].n) return ps[a].n > ps[b].n;
      return a < b;
    });
    // each weighted graph's largest weight: it sizes the slot rings of the
    // graph's group in the memory estimate below
    std::vector<uint32_t> mw(count, 1u);
    {
      std::vector<const fl_problem *> wp;
      for (uint32_t i : ok) wp.push_back(&ps[i]);
      fl::ensure_host_status(dc);
      if (!dc.arena.fixed()) dc.arena.reserve(((size_t)ok.size() + 1) * (sizeof(fl::WeightDesc) + 4) + 4096);
      dc.arena.reset();
      fl::Ctx c;
      c.s = (hipStream_t)stream;
      c.arena = &dc.arena;
      c.h_status = dc.h_status;
      const std::vector<uint32_t> m1 = fl::batch_max_weights(c, wp.data(), (uint32_t)wp.size());
      for (size_t t = 0; t < ok.size(); ++t) mw[ok[t]] = m1[t];
    }
    size_t free_b = 0, total_b = 0;
    FL_HIP(hipMemGetInfo(&free_b, &total_b));
    int devb = 0;
    FL_HIP(hipGetDevice(&devb));
    size_t held = dc.arena.capacity();
    for (int w = 0; w < fl::BATCH_WORKERS; ++w) held += fl::g_pool[devb].dc[w].arena.capacity();
    const size_t budget = (size_t)((double)(free_b + held) * 0.6);
    size_t i0 = 0;
    while (i0 < ok.size()) {
      const fl_params &P0 = prms[ok[i0]];
      size_t i1 = i0;
      uint64_t N = 0, M = 0;
      uint32_t nmax = 1, wmax = 1;
      bool wt = false;
      while (i1 < ok.size()) {
        const uint32_t j = ok[i1];
        const fl_params &Pj = prms[j];
        if (Pj.k != P0.k || Pj.eps != P0.eps || Pj.flags != P0.flags) break;
        const uint64_t N2 = N + ps[j].n, M2 = M + ps[j].n_arcs;
        const uint32_t nm2 = std::max(nmax, ps[j].n);
        const bool wt2 = wt || ps[j].w != nullptr;
        // a weight beyond MAX_W fails the group's validation; until then it
        // counts as MAX_W
        const uint32_t wm2 = std::min(std::max(wmax, ps[j].w ? mw[j] : 1u), fl::MAX_W);
        const uint32_t cap = fl::ads_capacity(nm2, P0.k);
        const size_t need = fl::estimate_bytes((uint32_t)std::min<uint64_t>(N2, 0xFFFFFFFEull), M2, N2, P0.k, cap,
                                               wt2 ? wm2 + 1 : 2) +
                            fl::union_bytes((uint32_t)(i1 - i0 + 1), N2, M2, wt2) +
                            ((P0.flags & FL_FLAG_DIRECTED) ? fl::transpose_bytes((uint32_t)std::min<uint64_t>(
                                                                 N2, 0xFFFFFFFEull), M2, wt2)
                                                           : 0);
        if (i1 > i0 && (need > budget || N2 >= 0x7FFFFFFFull || i1 - i0 >= 65535)) break;
        N = N2;
        M = M2;
        nmax = nm2;
        wmax = wm2;
        wt = wt2;
        ++i1;
      }
      std::vector<const fl_problem *> gp;
      std::vector<const fl_params *> gr;
      std::vector<fl_result *> go;
      for (size_t t = i0; t < i1; ++t) {
        gp.push_back(&ps[ok[t]]);
        gr.push_back(&prms[ok[t]]);
        go.push_back(&outs[ok[t]]);
      }
      std::vector<int> grc(gp.size(), FL_OK);
      const int P = (int)std::min<size_t>(fl::BATCH_WORKERS, gp.size());
      if (P <= 1) {
        try {
          fl::solve_group(gp.data(), gr.data(), go.data(), (uint32_t)gp.size(), (hipStream_t)stream, dc, grc);
        } catch (fl::Error &e) {
          grc.assign(gp.size(), e.code);
        }
      } else {
        // largest first onto the least loaded worker (elements are in
        // decreasing n already); each worker keeps its elements in order
        std::vector<std::vector<size_t>> part(P);
        std::vector<uint64_t> load(P, 0);
        for (size_t t = 0; t < gp.size(); ++t) {
          const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          part[w].push_back(t);
          load[w] += (uint64_t)gp[t]->n + gp[t]->n_arcs / 8;
        }
        int dev = 0;
        FL_HIP(hipGetDevice(&dev));
        fl::BatchPool &pool = fl::g_pool[dev];
        hipEvent_t ready;
        FL_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        FL_HIP(hipEventRecord(ready, (hipStream_t)stream));  // inputs written on the caller's stream
        std::vector<std::thread> th;
        for (int w = 0; w < P; ++w) {
          th.emplace_back([&, w]() {
            std::vector<const fl_problem *> sp;
            std::vector<const fl_params *> sr;
            std::vector<fl_result *> so;
            for (size_t t : part[w]) {
              sp.push_back(gp[t]);
              sr.push_back(gr[t]);
              so.push_back(go[t]);
            }
            std::vector<int> src;
            try {
              FL_HIP(hipSetDevice(dev));
              std::lock_guard<std::mutex> wl(pool.dc[w].mu);
              if (!pool.st[w]) FL_HIP(hipStreamCreateWithFlags(&pool.st[w], hipStreamNonBlocking));
              FL_HIP(hipStreamWaitEvent(pool.st[w], ready, 0));
              fl::solve_group(sp.data(), sr.data(), so.data(), (uint32_t)sp.size(), pool.st[w], pool.dc[w], src);
            } catch (fl::Error &e) {
              src.assign(sp.size(), e.code);
            } catch (std::bad_alloc &) {
              src.assign(sp.size(), FL_ENOMEM);
            }
            for (size_t j = 0; j < part[w].size(); ++j) grc[part[w][j]] = src[j];
          });
        }
        for (auto &t : th) t.join();
        (void)hipEventDestroy(ready);
      }
      for (size_t t = i0; t < i1; ++t) rc[ok[t]] = grc[t - i0];
      i0 = i1;
    }
    int first = FL_OK;
    for (uint32_t i = 0; i < count; ++i) {
      outs[i].status = rc[i];
      if (rc[i] != FL_OK) outs[i].n_open = 0;
      if (rc[i] != FL_OK && first == FL_OK) first = rc[i];
    }
    return first;
  } catch (fl::Error &e) {
    return e.code;
  } catch (std::bad_alloc &) {
    return FL_ENOMEM;
  }
}

int fl_ads_build(const fl_problem *p, const fl_params *prm, fl_sketch **out, void *stream) {
  if (!out) return FL_EINVAL;
  *out = nullptr;
  try {
    int rc = fl::check_params(p, prm);
    if (rc) return rc;
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    fl::ensure_host_status(dc);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t n = p->n;
    const uint32_t cap0 = fl::ads_capacity(n, prm->k);
    const bool directed = (prm->flags & FL_FLAG_DIRECTED) != 0;
    const size_t tr = directed ? fl::transpose_bytes(n, p->n_arcs, p->w != nullptr) : 0;
    dc.arena.reserve(fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, 2) + tr);
    dc.arena.reset();
    fl::Ctx c;
    c.s = s;
    c.arena = &dc.arena;
    c.h_status = dc.h_status;
    uint32_t max_w = 1, max_c = 0;
    fl_problem q = *p;
    q.fac_cost = nullptr;
    rc = fl::validate_graph(c, &q, directed, &max_w, &max_c);
    if (rc) return rc;
    if ((uint64_t)(n - 1) * (p->w ? max_w : 1u) >= 0xFFFFFFFFull) return FL_ERANGE;
    if (p->w && max_w > fl::MAX_W) return FL_ENOTIMPL;
    const uint32_t NS = (p->w ? max_w : 1u) + 1;
    if (fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, NS) + tr > dc.arena.capacity()) {
      dc.arena.reserve(fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, NS) + tr);
      dc.arena.reset();
      rc = fl::validate_graph(c, &q, directed, &max_w, &max_c);
      if (rc) return rc;
    }
    fl::Graph g{n, p->n_arcs, p->row_ptr, p->col, p->w, p->w ? max_w : 1u};
    fl::set_in_arcs(c, g, directed);
    fl::SegInfo hseg = fl::seg_info(0, n, prm->seed);
    fl::SegInfo *seg = c.arena->get<fl::SegInfo>(1);
    FL_HIP(hipMemcpyAsync(seg, &hseg, sizeof(hseg), hipMemcpyHostToDevice, s));
    fl::AdsConfig acfg{prm->k, nullptr, seg, prm->flags, n, nullptr, nullptr, n};
    fl::AdsOut ads;
    rc = fl::ads_build(c, g, acfg, ads);
    if (rc) return rc;
    uint64_t *off_tmp = c.arena->get<uint64_t>((size_t)n + 1);
    fl::scan_u32_to_u64(c, ads.cnt, off_tmp, n);
    FL_HIP(hipMemcpyAsync(c.h_status, off_tmp + n, 8, hipMemcpyDeviceToHost, s));
    c.sync();
    const uint64_t total = c.h_status[0];
    fl_sketch *sk = new fl_sketch();
    FL_HIP(hipGetDevice(&sk->device));
    sk->n = n;
    sk->k = prm->k;
    sk->total = total;
    const size_t bytes = ((size_t)n + 1) * 8 + total * 12 + 1024;
    sk->mem = fl::dev_alloc(bytes);
    if (!sk->mem) {
      delete sk;
      return FL_ENOMEM;
    }
    char *m = static_cast<char *>(sk->mem);
    sk->off = reinterpret_cast<uint64_t *>(m);
    sk->rank = reinterpret_cast<uint32_t *>(m + ((size_t)n + 1) * 8);
    sk->dist = sk->rank + total;
    sk->thr = sk->dist + total;
    FL_HIP(hipMemcpyAsync(sk->off, off_tmp, ((size_t)n + 1) * 8, hipMemcpyDeviceToDevice, s));
    fl::ads_export(c, g, ads, sk->off, sk->rank, sk->dist, sk->thr);
    c.sync();
    *out = sk;
    return FL_OK;
  } catch (fl::Error &e) {
    return e.code;
  } catch (std::bad_alloc &) {
    return FL_ENOMEM;
  }
}

int fl_sketch_view(const fl_sketch *s, fl_sketch_view_t *v) {
  if (!s || !v) return FL_EINVAL;
  v->n = s->n;
  v->k = s->k;
  v->total = s->total;
  v->off = s->off;
  v->rank = s->rank;
  v->dist = s->dist;
  v->thresh = s->thr;
  return FL_OK;
}

void fl_sketch_free(fl_sketch *s) {
  if (!s) return;
  fl::dev_free(s->mem);
  delete s;
}

uint32_t fl_rank_of(uint32_t v, uint64_t seed) { return fl::perm_fwd(v, fl::perm_key(seed, 1)); }
uint32_t fl_priority_of(uint32_t v, uint64_t seed) { return fl::perm_fwd(v, fl::perm_key(seed, 2)); }

const char *fl_strerror(int code) {
  switch (code) {
    case FL_OK: return "ok";
    case FL_EINVAL: return "invalid argument or malformed graph";
    case FL_ERANGE: return "distances or costs could overflow 32 bits";
    case FL_ENOMEM: return "workspace does not fit";
    case FL_EHIP: return "HIP runtime error";
    case FL_EBUSY: return "busy";
    case FL_ENOTIMPL: return "outside the limits of this library (k > 128, weight > 255, sketch capacity)";
    default: return "unknown error";
  }
}

int fl_last_hip_error(void) { return fl::g_last_hip.load(); }

int fl_server_create(uint64_t hbm_budget_bytes, uint32_t slots, fl_server **out) {
  if (!out) return FL_EINVAL;
  *out = nullptr;
  try {
    fl_server *sv = new fl_server();
    fl::Server &S = sv->s;
    FL_HIP(hipGetDevice(&S.device));
    if (hbm_budget_bytes == 0) {
      size_t fr = 0, tot = 0;
      FL_HIP(hipMemGetInfo(&fr, &tot));
      hbm_budget_bytes = (uint64_t)((double)fr * 0.6);
    }
    S.budget = (size_t)hbm_budget_bytes;
    const uint32_t ns = slots ? slots : 3u;
    for (uint32_t i = 0; i < ns; ++i) {
      fl::Slot *sl = new fl::Slot();
      sl->srv = &S;
      FL_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
      fl::ensure_host_status(sl->dc);
      S.slots.push_back(sl);
    }
    for (fl::Slot *sl : S.slots) sl->th = std::thread(fl::slot_main, sl);
    fl::g_servers.fetch_add(1);
    *out = sv;
    return FL_OK;
  } catch (fl::Error &e) {
    return e.code;
  } catch (std::bad_alloc &) {
    return FL_ENOMEM;
  }
}

int fl_server_submit(fl_server *sv, const fl_problem *p, const fl_params *prm, fl_result *out, uint64_t *ticket) {
  if (!sv || !ticket) return FL_EINVAL;
  int pc = fl::check_params(p, prm);
  if (pc) return pc;
  if (!p->fac_cost || !out || !out->open || !out->assign) return FL_EINVAL;
  fl::Server &S = sv->s;
  fl::Request *r = new fl::Request();
  r->p = p;
  r->prm = prm;
  r->out = out;
  std::vector<fl::Request *> one(1, r);
  r->bytes = fl::group_bytes(one);
  if (r->bytes > S.budget) {
    delete r;
    return FL_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stop) {
      delete r;
      return FL_EBUSY;
    }
    r->ticket = S.next_ticket++;
    S.reqs[r->ticket] = r;
    S.queue.push_back(r);
    *ticket = r->ticket;
  }
  S.cv_work.notify_one();
  return FL_OK;
}

static int server_finish(fl::Server &S, uint64_t ticket, int *status, bool block) {
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.reqs.find(ticket);
  if (it == S.reqs.end()) return FL_EINVAL;
  fl::Request *r = it->second;
  while (!r->done) {
    if (!block) return FL_EBUSY;
    S.cv_done.wait(lk);
  }
  if (status) *status = r->status;
  S.reqs.erase(it);
  delete r;
  return FL_OK;
}

int fl_server_poll(fl_server *sv, uint64_t ticket, int *status) {
  if (!sv) return FL_EINVAL;
  return server_finish(sv->s, ticket, status, false);
}

int fl_server_wait(fl_server *sv, uint64_t ticket, int *status) {
  if (!sv) return FL_EINVAL;
  return server_finish(sv->s, ticket, status, true);
}

void fl_server_destroy(fl_server *sv) {
  if (!sv) return;
  fl::Server &S = sv->s;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv_work.notify_all();
  for (fl::Slot *sl : S.slots) {
    if (sl->th.joinable()) sl->th.join();
    (void)hipStreamDestroy(sl->stream);
    sl->dc.release_all();
    delete sl;
  }
  for (auto &kv : S.reqs) delete kv.second;
  delete sv;
  fl::g_servers.fetch_sub(1);
}

int fl_set_allocator(fl_alloc_fn alloc, fl_free_fn free_fn, void *ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return FL_EINVAL;
  if (fl::g_servers.load() > 0) return FL_EBUSY;
  // cached workspaces go back through the hooks they came from
  for (int d = 0; d < 64; ++d) {
    {
      std::lock_guard<std::mutex> lk(fl::g_cache[d].mu);
      fl::g_cache[d].arena.release();
    }
    for (int w = 0; w < fl::BATCH_WORKERS; ++w) {
      std::lock_guard<std::mutex> lk(fl::g_pool[d].dc[w].mu);
      fl::g_pool[d].dc[w].arena.release();
    }
  }
  std::lock_guard<std::mutex> lk(fl::g_hooks_mu);
  fl::g_hooks = fl::AllocHooks{alloc, free_fn, alloc ? ctx : nullptr};
  return FL_OK;
}

void fl_release_workspace(void) {
  try {
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    dc.arena.release();
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64)
      for (int w = 0; w < fl::BATCH_WORKERS; ++w) {
        std::lock_guard<std::mutex> wl(fl::g_pool[dev].dc[w].mu);
        fl::g_pool[dev].dc[w].arena.release();
      }
  } catch (...) {
  }
}

}  // extern "C"
