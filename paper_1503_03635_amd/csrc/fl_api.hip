// fl_api.hip -- the C ABI (include/fl.h): parameter checks, workspace
// management and the solve driver that chains the phases
//   validate -> ranks/sketches -> gamma and ladder -> opening loop -> MIS ->
//   assignment -> objective.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
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

void Arena::reserve(size_t bytes) {
  bytes = (bytes + (size_t(1) << 21) - 1) & ~((size_t(1) << 21) - 1);
  if (bytes <= cap_) return;
  release();
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (std::getenv("FL_DEBUG")) std::fprintf(stderr, "[fl] workspace %zu bytes: %s\n", bytes, hipGetErrorString(e));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{FL_ENOMEM};
  }
  base_ = static_cast<char *>(p);
  cap_ = bytes;
  used_ = 0;
}
void Arena::release() {
  if (base_) (void)hipFree(base_);
  base_ = nullptr;
  cap_ = used_ = 0;
}

struct DeviceCache {
  std::mutex mu;
  Arena arena;
  uint64_t *h_status = nullptr;
};
static DeviceCache g_cache[64];

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
// served clients, gamma, counts.  ctr: [0..63] nC, [64..127] nCeff,
// [128..191] nUF0, [192..255] max gamma
__global__ void k_clients(uint32_t n, const uint8_t *is_client, const uint64_t *gl, const uint32_t *fac_cost,
                          uint8_t *ceff, uint64_t *ctr) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool cl = false, ce = false, uf = false;
  uint64_t gmax = 0;
  if (v < n) {
    cl = is_client ? is_client[v] != 0 : true;
    ce = cl && gl[v] != INF64;
    uf = ce && fac_cost[v] != FL_NOT_FACILITY;
    ceff[v] = ce ? 1 : 0;
    if (ce) gmax = gl[v] >> 32;
  }
  const uint64_t a = __popcll(__ballot(cl)), b = __popcll(__ballot(ce)), d = __popcll(__ballot(uf));
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const uint64_t o = __shfl_xor(gmax, s, WAVE);
    gmax = o > gmax ? o : gmax;
  }
  if (lane_id() == 0) {
    const int st = blockIdx.x & 63;
    atomicAdd((unsigned long long *)&ctr[st], (unsigned long long)a);
    atomicAdd((unsigned long long *)&ctr[64 + st], (unsigned long long)b);
    atomicAdd((unsigned long long *)&ctr[128 + st], (unsigned long long)d);
    atomicMax((unsigned long long *)&ctr[192 + st], (unsigned long long)gmax);
  }
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
// assignment outputs and the objective.  ctr: [0..63] cost, [64..127]
// n_open, [128..191] n_guard
__global__ void k_assign_out(uint32_t n, const uint8_t *ceff, const uint64_t *lab, const uint8_t *open,
                             const uint32_t *fac_cost, const uint32_t *orung, uint32_t *assign,
                             uint32_t *dist, uint64_t *ctr) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t cost = 0, no = 0, ng = 0;
  if (v < n) {
    if (ceff[v]) {
      const uint64_t L = lab[v];
      assign[v] = (uint32_t)(L & 0xFFFFFFFFu);
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
    }
    if (orung[v] == FL_RUNG_GUARD) ng = 1;
  }
  cost = wave_sum_u64(cost);
  no = wave_sum_u64(no);
  ng = wave_sum_u64(ng);
  if (lane_id() == 0) {
    const int st = blockIdx.x & 63;
    atomicAdd((unsigned long long *)&ctr[st], (unsigned long long)cost);
    atomicAdd((unsigned long long *)&ctr[64 + st], (unsigned long long)no);
    atomicAdd((unsigned long long *)&ctr[128 + st], (unsigned long long)ng);
  }
}

static void read_u64_fields(Ctx &c, const uint64_t *d, int fields, std::vector<uint64_t> &sum,
                            bool max_last = false) {
  std::vector<uint64_t> h((size_t)fields * 64);
  FL_HIP(hipMemcpyAsync(h.data(), d, h.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  sum.assign(fields, 0);
  for (int f = 0; f < fields; ++f)
    for (int s = 0; s < 64; ++s) {
      const uint64_t x = h[(size_t)f * 64 + s];
      if (max_last && f == fields - 1) sum[f] = x > sum[f] ? x : sum[f];
      else sum[f] += x;
    }
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
  const size_t later = (size_t)NS * n * 8 + (size_t)n * 160 + (size_t)nF * 96;  // opening loop, MIS, assignment
  b += ads > later ? ads : later;
  b += (size_t)64 << 20;                   // counters, scans
  return b;
}

static double ms_between(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return (double)ms;
}

static int solve_one(const fl_problem *p, const fl_params *prm, fl_result *out, hipStream_t s,
                     DeviceCache &dc) {
  int rc = check_params(p, prm);
  if (rc) return rc;
  if (!p->fac_cost || !out || !out->open || !out->assign) return FL_EINVAL;
  ensure_host_status(dc);
  const uint32_t n = p->n;
  const uint32_t cap0 = ads_capacity(n, prm->k);
  // facilities are counted after validation; reserve for all vertices first
  dc.arena.reserve(estimate_bytes(n, p->n_arcs, n, prm->k, cap0, 2));
  dc.arena.reset();
  Ctx c;
  c.s = s;
  c.arena = &dc.arena;
  c.h_status = dc.h_status;

  hipEvent_t ev[8];
  for (auto &e : ev) FL_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(e[i]);
    }
  } evg{ev};
  FL_HIP(hipEventRecord(ev[0], s));

  uint32_t max_w = 1, max_c = 0;
  rc = validate_graph(c, p, &max_w, &max_c);
  if (rc) return rc;
  const uint64_t bound = (uint64_t)(n - 1) * (p->w ? max_w : 1u) + max_c;
  if (bound >= 0xFFFFFFFFull) return FL_ERANGE;
  if (p->w && max_w > MAX_W) return FL_ENOTIMPL;
  Graph g{n, p->n_arcs, p->row_ptr, p->col, p->w, p->w ? max_w : 1u};
  const uint32_t NS = g.max_w + 1;
  FL_HIP(hipEventRecord(ev[1], s));

  // facilities
  uint32_t *flag = c.arena->get<uint32_t>(n);
  uint64_t *pos = c.arena->get<uint64_t>((size_t)n + 1);
  uint32_t *fac_list = c.arena->get<uint32_t>(n);
  uint32_t *fac_idx = c.arena->get<uint32_t>(n);
  const uint32_t vb = (uint32_t)ceil_div(n, 256);
  k_fac_flags<<<vb, 256, 0, s>>>(n, p->fac_cost, flag);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, flag, pos, n);
  k_fac_index<<<vb, 256, 0, s>>>(n, flag, pos, fac_list, fac_idx);
  FL_LAUNCH_CHECK();
  FL_HIP(hipMemcpyAsync(c.h_status, pos + n, 8, hipMemcpyDeviceToHost, s));
  c.sync();
  const uint32_t nF = (uint32_t)c.h_status[0];
  // re-reserve now that the sizes are known (keeps what is allocated so far
  // valid only if no reallocation happens; reserve before any use instead)
  if (estimate_bytes(n, p->n_arcs, nF, prm->k, cap0, NS) > dc.arena.capacity()) {
    dc.arena.reserve(estimate_bytes(n, p->n_arcs, nF, prm->k, cap0, NS));
    return solve_one(p, prm, out, s, dc);  // restart with the larger arena
  }

  // sketches
  AdsConfig acfg{prm->k, prm->seed, prm->flags, nF, fac_idx, fac_list};
  AdsOut ads;
  rc = ads_build(c, g, acfg, ads);
  if (rc) return rc;
  ads_totals(c, g, ads.cnt, &out->stats.relax_alg, &out->stats.ads_entries);
  out->stats.ads_rounds = ads.rounds;
  out->stats.relax_exec = ads.relax_exec;
  out->stats.ms_ads_kernel = ads.kernel_ms;
  out->stats.ads_kernel_launches = ads.launches;
  FL_HIP(hipEventRecord(ev[2], s));

  // gamma (Sec. 4.1) and served clients
  uint64_t *gl = c.arena->get<uint64_t>(n);
  uint8_t *ceff = c.arena->get<uint8_t>(n);
  uint64_t *ctr = c.arena->get<uint64_t>(256);
  k_gamma_init<<<vb, 256, 0, s>>>(n, p->fac_cost, gl);
  FL_LAUNCH_CHECK();
  SsspWork wk;
  sssp_alloc(c, wk, n);
  sssp_run(c, g, gl, fac_list, nF, wk, 0);
  fill_u64(c, ctr, 256, 0);
  k_clients<<<vb, 256, 0, s>>>(n, p->is_client, gl, p->fac_cost, ceff, ctr);
  FL_LAUNCH_CHECK();
  std::vector<uint64_t> cs;
  read_u64_fields(c, ctr, 4, cs, true);
  const uint64_t nC = cs[0], nCeff = cs[1], nUF0 = cs[2], gamma = cs[3];
  out->stats.gamma = gamma;
  out->n_unreachable = (uint32_t)(nC - nCeff);
  const double one_eps = 1.0 + prm->eps;
  std::vector<double> lad(1, 0.0);
  if (nF > 0 && nCeff > 0) {
    const double M = (double)((uint64_t)nF * nCeff);
    lad[0] = ((double)gamma / (M * M)) * one_eps;
  }
  lad.push_back(lad[0] * one_eps);
  out->stats.alpha0 = lad[0];
  FL_HIP(hipEventRecord(ev[3], s));

  // opening loop
  uint32_t *orung = out->open_rung ? out->open_rung : c.arena->get<uint32_t>(n);
  uint32_t *frz = out->freeze_rung ? out->freeze_rung : c.arena->get<uint32_t>(n);
  double *qf = c.arena->get<double>(nF ? nF : 1);
  OpenIn oi{&g, nF, fac_list, fac_idx, p->fac_cost, &ads, perm_key(prm->seed, 1), ceff, nCeff, nUF0, gl,
            prm->eps, &lad};
  OpenOut oo{orung, frz, qf};
  rc = open_phase(c, oi, oo);
  if (rc) return rc;
  out->stats.rungs = oo.rungs;
  if (out->q) {
    fill_f64(c, out->q, n, 0.0);
    if (nF) {
      k_scatter_q<<<(uint32_t)ceil_div(nF, 256), 256, 0, s>>>(nF, fac_list, qf, out->q);
      FL_LAUNCH_CHECK();
    }
  }
  FL_HIP(hipEventRecord(ev[4], s));

  // MIS per rung
  MisIn mi{&g, oo.rungs, &lad, prm->eps, orung, frz, perm_key(prm->seed, 2)};
  uint32_t mis_rounds = 0;
  rc = mis_phase(c, mi, out->open, &mis_rounds);
  if (rc) return rc;
  out->stats.mis_rounds = mis_rounds;
  FL_HIP(hipEventRecord(ev[5], s));

  // assignment and objective (Sec. 3.1)
  uint64_t *al = c.arena->get<uint64_t>(n);
  k_assign_init<<<vb, 256, 0, s>>>(n, out->open, al, flag);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, flag, pos, n);
  uint32_t *slist = c.arena->get<uint32_t>(n);
  k_compact_u32<<<vb, 256, 0, s>>>(n, flag, pos, slist);
  FL_LAUNCH_CHECK();
  FL_HIP(hipMemcpyAsync(c.h_status, pos + n, 8, hipMemcpyDeviceToHost, s));
  c.sync();
  const uint32_t nS = (uint32_t)c.h_status[0];
  sssp_run(c, g, al, slist, nS, wk, 0);
  fill_u64(c, ctr, 256, 0);
  k_assign_out<<<vb, 256, 0, s>>>(n, ceff, al, out->open, p->fac_cost, orung, out->assign, out->dist, ctr);
  FL_LAUNCH_CHECK();
  read_u64_fields(c, ctr, 3, cs);
  out->total_cost = cs[0];
  out->n_open = (uint32_t)cs[1];
  out->stats.n_guard = (uint32_t)cs[2];
  FL_HIP(hipEventRecord(ev[6], s));
  FL_HIP(hipEventSynchronize(ev[6]));
  out->stats.ms_validate = ms_between(ev[0], ev[1]);
  out->stats.ms_ads = ms_between(ev[1], ev[2]);
  out->stats.ms_gamma = ms_between(ev[2], ev[3]);
  out->stats.ms_open = ms_between(ev[3], ev[4]);
  out->stats.ms_mis = ms_between(ev[4], ev[5]);
  out->stats.ms_assign = ms_between(ev[5], ev[6]);
  out->stats.ms_total = ms_between(ev[0], ev[6]);
  out->stats.workspace_bytes = c.arena->used();
  return FL_OK;
}

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
  try {
    if (out) std::memset(&out->stats, 0, sizeof(out->stats));
    int pc = fl::check_params(p, prm);
    if (pc) return pc;
    if (!p->fac_cost || !out || !out->open || !out->assign) return FL_EINVAL;
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    int rc = fl::solve_one(p, prm, out, (hipStream_t)stream, dc);
    if (rc != FL_OK && out) out->n_open = 0;
    return rc;
  } catch (fl::Error &e) {
    if (out) out->n_open = 0;
    return e.code;
  } catch (std::bad_alloc &) {
    return FL_ENOMEM;
  }
}

int fl_solve_batch(const fl_problem *ps, const fl_params *prms, fl_result *outs, uint32_t count,
                   void *stream) {
  if (count && (!ps || !prms || !outs)) return FL_EINVAL;
  int first = FL_OK;
  for (uint32_t i = 0; i < count; ++i) {
    int rc = fl_solve(&ps[i], &prms[i], &outs[i], stream);
    if (rc != FL_OK && first == FL_OK) first = rc;
  }
  return first;
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
    dc.arena.reserve(fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, 2));
    dc.arena.reset();
    fl::Ctx c;
    c.s = s;
    c.arena = &dc.arena;
    c.h_status = dc.h_status;
    uint32_t max_w = 1, max_c = 0;
    fl_problem q = *p;
    q.fac_cost = nullptr;
    rc = fl::validate_graph(c, &q, &max_w, &max_c);
    if (rc) return rc;
    if ((uint64_t)(n - 1) * (p->w ? max_w : 1u) >= 0xFFFFFFFFull) return FL_ERANGE;
    if (p->w && max_w > fl::MAX_W) return FL_ENOTIMPL;
    const uint32_t NS = (p->w ? max_w : 1u) + 1;
    if (fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, NS) > dc.arena.capacity()) {
      dc.arena.reserve(fl::estimate_bytes(n, p->n_arcs, n, prm->k, cap0, NS));
      dc.arena.reset();
      rc = fl::validate_graph(c, &q, &max_w, &max_c);
      if (rc) return rc;
    }
    fl::Graph g{n, p->n_arcs, p->row_ptr, p->col, p->w, p->w ? max_w : 1u};
    fl::AdsConfig acfg{prm->k, prm->seed, prm->flags, n, nullptr, nullptr};
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
    if (hipMalloc(&sk->mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
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
  (void)hipFree(s->mem);
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
    case FL_ENOTIMPL: return "outside the limits of this build (k > 64, weight > 255, sketch capacity)";
    default: return "unknown error";
  }
}

int fl_last_hip_error(void) { return fl::g_last_hip.load(); }

void fl_release_workspace(void) {
  try {
    fl::DeviceCache &dc = fl::cache_for_current();
    std::lock_guard<std::mutex> lk(dc.mu);
    dc.arena.release();
  } catch (...) {
  }
}

}  // extern "C"
