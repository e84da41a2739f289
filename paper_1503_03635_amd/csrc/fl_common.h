// fl_common.h -- internal definitions shared by the HIP sources of the
// library: wave64 helpers, the seeded rank bijection, exact fixed-point
// helpers for the HIP-estimator sums, and the workspace arena.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/fl.h"

namespace fl {

constexpr int WAVE = 64;
constexpr uint32_t INF32 = 0xFFFFFFFFu;
constexpr uint64_t INF64 = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t MAX_K = 128;  // the running bottom-k set: at most two registers per lane
constexpr uint32_t MAX_W = 255;      // largest edge weight handled by the slot ring
constexpr uint32_t MAX_CAP = 65535;  // largest per-vertex sketch capacity
constexpr int NCTR = 1024;           // strided counters (spread atomics over addresses)

// ---------------------------------------------------------------------------
// Error plumbing
// ---------------------------------------------------------------------------
struct Error {
  int code;
};
void set_last_hip_error(int e);

#define FL_HIP(call)                                                \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) {                                         \
      ::fl::set_last_hip_error((int)e_);                            \
      throw ::fl::Error{FL_EHIP};                                   \
    }                                                               \
  } while (0)

#define FL_LAUNCH_CHECK() FL_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Seeded bijection on 32-bit ids.  Ranks r(v) and MIS priorities pi(f) are
// "hashes" of the vertex id (Alg. 1; Sec. 4.3).  Both are bijections here:
// two rounds of the MurmurHash3 32-bit finaliser (public domain), each after
// an xor with a 32-bit key; the two keys of a stream are the halves of
// SplitMix64 (Vigna, public domain) applied to seed^1 (ranks) or seed^2
// (priorities).  All steps are invertible, so a rank maps back to its vertex.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr uint32_t modinv32(uint32_t c) {
  uint32_t x = c;
  for (int i = 0; i < 5; ++i) x *= 2u - c * x;
  return x;
}
constexpr uint32_t MUR_C1 = 0x85ebca6bu, MUR_C2 = 0xc2b2ae35u;
constexpr uint32_t MUR_C1_INV = modinv32(MUR_C1), MUR_C2_INV = modinv32(MUR_C2);
static_assert(MUR_C1 * MUR_C1_INV == 1u, "inverse");
static_assert(MUR_C2 * MUR_C2_INV == 1u, "inverse");

__host__ __device__ inline uint32_t murmur_fmix(uint32_t h) {
  h ^= h >> 16;
  h *= MUR_C1;
  h ^= h >> 13;
  h *= MUR_C2;
  h ^= h >> 16;
  return h;
}
__host__ __device__ inline uint32_t murmur_unfmix(uint32_t h) {
  h ^= h >> 16;                      // x ^ (x >> 16) is its own inverse on 32 bits
  h *= MUR_C2_INV;
  h ^= (h >> 13) ^ (h >> 26);        // inverse of x ^ (x >> 13)
  h *= MUR_C1_INV;
  h ^= h >> 16;
  return h;
}

struct PermKey {
  uint32_t k1, k2;
};
__host__ __device__ inline PermKey perm_key(uint64_t seed, uint64_t stream) {
  uint64_t s = splitmix64(seed ^ stream);
  return PermKey{(uint32_t)s, (uint32_t)(s >> 32)};
}
__host__ __device__ inline uint32_t perm_fwd(uint32_t v, PermKey k) {
  return murmur_fmix(murmur_fmix(v ^ k.k1) ^ k.k2);
}
__host__ __device__ inline uint32_t perm_inv(uint32_t r, PermKey k) {
  return murmur_unfmix(murmur_unfmix(r) ^ k.k2) ^ k.k1;
}

// ---------------------------------------------------------------------------
// Several independent graphs are solved together as one disjoint union:
// vertex v of graph g is vertex base + v of the union.  Ranks, priorities and
// the id buckets of the level prune use the local id with the graph's own
// keys, and local order is union order inside a graph, so every graph gets
// exactly the result it gets alone.  A single graph is the union of one
// (gid == nullptr, base 0).
// ---------------------------------------------------------------------------
struct SegInfo {
  uint32_t base, n;
  PermKey rk, pk;   // rank (stream 1) and MIS-priority (stream 2) keys
  uint32_t bshift;  // level-prune id bucket: local id >> bshift < 64
  uint32_t pad;
  uint64_t seed;    // the graph's seed (Luby's MIS draws per-round keys from it)
};

struct RankMap {
  PermKey rk;
  uint32_t base, bshift;
};
__host__ __device__ inline uint32_t seg_of(const uint32_t *gid, uint32_t v) { return gid ? gid[v] : 0u; }
__host__ __device__ inline RankMap rank_map(const SegInfo &s) { return RankMap{s.rk, s.base, s.bshift}; }
__host__ __device__ inline uint32_t rank_of(uint32_t id, const RankMap &m) { return perm_fwd(id - m.base, m.rk); }
__host__ __device__ inline uint32_t id_of(uint32_t r, const RankMap &m) { return perm_inv(r, m.rk) + m.base; }
__host__ __device__ inline uint32_t bucket_of(uint32_t id, const RankMap &m) { return (id - m.base) >> m.bshift; }
inline uint32_t bucket_shift(uint32_t n) {
  uint32_t bits = 0;
  while (bits < 32 && (1ull << bits) < (uint64_t)n) ++bits;
  return bits > 6 ? bits - 6 : 0;  // 64 buckets
}
inline SegInfo seg_info(uint32_t base, uint32_t n, uint64_t seed) {
  return SegInfo{base, n, perm_key(seed, 1), perm_key(seed, 2), bucket_shift(n), 0, seed};
}

// ---------------------------------------------------------------------------
// Exact sums of HIP-estimator weights.  A weight a = fl(2^32 / T) lies in
// [1, 2^32], so a * 2^52 is an integer below 2^85.  It is split at bit 40 into
// hi (< 2^45) and lo (< 2^40); sums of fewer than 2^16 such parts fit in 64
// bits, so a sum over a sketch is exact, and it is rounded to double once.
// ---------------------------------------------------------------------------
__host__ __device__ inline double hip_weight(uint32_t T) {
  // T == 0 encodes 2^32 (fewer than k earlier entries): weight 1
  return T == 0 ? 1.0 : 4294967296.0 / (double)T;
}
struct Fix52 {
  uint64_t hi, lo;
};
__host__ __device__ inline Fix52 fix52_of(double a) {
  uint64_t bits;
  memcpy(&bits, &a, sizeof(bits));
  int e = (int)((bits >> 52) & 0x7FF) - 1023;            // 0..32 for a in [1, 2^32]
  uint64_t mant = (bits & ((1ull << 52) - 1)) | (1ull << 52);
  Fix52 r;
  r.lo = (mant << e) & ((1ull << 40) - 1);
  r.hi = mant >> (40 - e);
  return r;
}
// round-to-nearest-even of (hi * 2^40 + lo) to double, then scaled by 2^-52
__host__ __device__ inline double fix52_to_double(uint64_t hi, uint64_t lo) {
  // 128-bit value V = hi * 2^40 + lo  (hi < 2^61, lo < 2^57)
  uint64_t vlo = (hi << 40);
  uint64_t vhi = hi >> 24;
  uint64_t s = vlo + lo;
  vhi += (s < vlo) ? 1 : 0;
  vlo = s;
  double d;
  if (vhi == 0) {
    if (vlo < (1ull << 53)) {
      d = (double)vlo;                                   // exact
    } else {
      int p = 63 - __builtin_clzll(vlo);                 // top bit, >= 53
      int sh = p - 52;
      uint64_t m = vlo >> sh;
      uint64_t rem = vlo & ((1ull << sh) - 1);
      uint64_t half = 1ull << (sh - 1);
      if (rem > half || (rem == half && (m & 1))) m++;
      d = ldexp((double)m, sh);
    }
  } else {
    int p = 64 + 63 - __builtin_clzll(vhi);              // top bit index
    int sh = p - 52;                                      // >= 12
    // m = V >> sh, rem = V mod 2^sh
    uint64_t m, rem, half;
    if (sh < 64) {
      m = (vlo >> sh) | (vhi << (64 - sh));
      rem = vlo & ((1ull << sh) - 1);
      half = 1ull << (sh - 1);
      bool up = rem > half || (rem == half && (m & 1));
      if (up) m++;
    } else {
      int s2 = sh - 64;
      m = vhi >> s2;
      uint64_t remhi = s2 ? (vhi & ((1ull << s2) - 1)) : 0;
      // compare (remhi, vlo) with half = 2^(sh-1)
      bool gt, eq;
      if (s2 == 0) {
        gt = vlo > (1ull << 63);
        eq = vlo == (1ull << 63);
      } else {
        uint64_t hh = 1ull << (s2 - 1);
        gt = remhi > hh || (remhi == hh && vlo > 0);
        eq = remhi == hh && vlo == 0;
      }
      if (gt || (eq && (m & 1))) m++;
    }
    d = ldexp((double)m, sh);
  }
  return ldexp(d, -52);
}

// ---------------------------------------------------------------------------
// Wave64 helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline uint32_t wave_scan_incl(uint32_t x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint32_t y = __shfl_up(x, d, WAVE);
    if (l >= d) x += y;
  }
  return x;
}
__device__ inline uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
  return x;
}
__device__ inline uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t y = __shfl_xor(x, d, WAVE);
    x = y < x ? y : x;
  }
  return x;
}
// number of set bits of mask below this lane
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
}

// Per-graph counters: field f of graph g, stripe s at [(g * nf + f) * stripes + s].
// Every lane of the wave calls; lanes with valid == false add nothing.  One
// atomic per wave when the valid lanes share a graph, one per lane otherwise.
__device__ inline void seg_add(unsigned long long *ctr, bool valid, uint32_t g, uint32_t f, uint32_t nf,
                               uint32_t stripes, uint64_t v) {
  const uint64_t vm = __ballot(valid);
  if (!vm) return;
  const uint32_t g0 = __shfl(g, __ffsll((long long)vm) - 1, WAVE);
  if (!__ballot(valid && g != g0)) {
    const uint64_t tot = wave_sum_u64(valid ? v : 0);
    if (lane_id() == 0 && tot) atomicAdd(&ctr[((size_t)g0 * nf + f) * stripes + blockIdx.x % stripes], tot);
  } else if (valid && v) {
    atomicAdd(&ctr[((size_t)g * nf + f) * stripes], (unsigned long long)v);
  }
}
__device__ inline void seg_add32(uint32_t *ctr, bool valid, uint32_t g, uint32_t f, uint32_t nf, uint32_t stripes,
                                 uint32_t v) {
  const uint64_t vm = __ballot(valid);
  if (!vm) return;
  const uint32_t g0 = __shfl(g, __ffsll((long long)vm) - 1, WAVE);
  if (!__ballot(valid && g != g0)) {
    const uint32_t tot = (uint32_t)wave_sum_u64(valid ? v : 0);
    if (lane_id() == 0 && tot) atomicAdd(&ctr[((size_t)g0 * nf + f) * stripes + blockIdx.x % stripes], tot);
  } else if (valid && v) {
    atomicAdd(&ctr[((size_t)g * nf + f) * stripes], v);
  }
}
__device__ inline uint32_t wave_max_u32(uint32_t x) { return ~wave_min_u32(~x); }
__device__ inline uint64_t shfl_u64(uint64_t x, int src) {
  const uint32_t lo = __shfl((uint32_t)x, src, WAVE), hi = __shfl((uint32_t)(x >> 32), src, WAVE);
  return ((uint64_t)hi << 32) | lo;
}
// wave-aggregated append of x to list (lanes with want)
__device__ inline void wave_push(uint32_t *list, uint32_t *count, bool want, uint32_t x) {
  const uint64_t m = __ballot(want);
  if (!m) return;
  const int lead = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == lead) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = __shfl(base, lead, WAVE);
  if (want) list[base + lanes_below(m)] = x;
}
// Frontier expansion: rows up to FLAT_MAX arcs are flattened over the wave
// (step c takes arcs c*64 .. c*64+63 of the concatenated rows, each lane
// finding its row by binary search over the running degree sum); longer rows
// go to a queue that a second kernel walks one row per wave.
constexpr uint32_t FLAT_MAX = 256;
// f(valid, arc, owner_lane) is called by every lane of the wave, converged.
template <class F>
__device__ inline void flat_arcs(bool light, uint64_t a0, uint64_t deg, F &&f) {
  const int lane = lane_id();
  const uint32_t d = light ? (uint32_t)deg : 0u;
  const uint32_t incl = wave_scan_incl(d);
  const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
  const uint32_t excl = incl - d;
  for (uint32_t c0 = 0; c0 < total; c0 += WAVE) {
    const uint32_t idx = c0 + lane;
    uint32_t pos = 0;  // first lane whose inclusive sum exceeds idx
#pragma unroll
    for (uint32_t s = 32; s >= 1; s >>= 1) {
      const uint32_t val = __shfl(incl, (int)(pos + s - 1), WAVE);
      if (val <= idx) pos += s;
    }
    const bool valid = idx < total;
    const uint64_t oa = shfl_u64(a0, (int)(valid ? pos : 0));
    const uint32_t oe = __shfl(excl, (int)(valid ? pos : 0), WAVE);
    f(valid, oa + (idx - oe), (int)(valid ? pos : 0));
  }
}
__device__ inline void seg_max(unsigned long long *ctr, bool valid, uint32_t g, uint32_t f, uint32_t nf,
                               uint32_t stripes, uint64_t v) {
  const uint64_t vm = __ballot(valid);
  if (!vm) return;
  const uint32_t g0 = __shfl(g, __ffsll((long long)vm) - 1, WAVE);
  if (!__ballot(valid && g != g0)) {
    uint64_t mx = valid ? v : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const uint64_t o = __shfl_xor(mx, d, WAVE);
      mx = o > mx ? o : mx;
    }
    if (lane_id() == 0 && mx) atomicMax(&ctr[((size_t)g0 * nf + f) * stripes + blockIdx.x % stripes], mx);
  } else if (valid && v) {
    atomicMax(&ctr[((size_t)g * nf + f) * stripes], (unsigned long long)v);
  }
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// A bump arena over one cached device allocation, or over a fixed buffer
// the arena does not own (attach): that one never grows, and running out of
// it throws FL_ENOMEM before any pointer past its end is handed out.
class Arena {
 public:
  void reserve(size_t bytes);
  void attach(char *base, size_t cap) {
    base_ = base;
    cap_ = cap;
    used_ = peak_ = 0;
    fixed_ = true;
  }
  bool fixed() const { return fixed_; }
  void reset() { used_ = 0; }
  void rewind(size_t mark) { used_ = mark; }
  template <class T>
  T *get(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (used_ + bytes > cap_) {
      if (std::getenv("FL_DEBUG"))
        std::fprintf(stderr, "[fl] arena exhausted: used %zu + %zu > cap %zu\n", used_, bytes, cap_);
      throw Error{FL_ENOMEM};
    }
    T *p = reinterpret_cast<T *>(base_ + used_);
    used_ += bytes;
    if (used_ > peak_) peak_ = used_;
    return p;
  }
  size_t used() const { return used_; }
  size_t capacity() const { return cap_; }
  void release();

 private:
  char *base_ = nullptr;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  bool fixed_ = false;
};

// Per-call context: stream, arena, pinned host scratch for status readbacks.
struct Ctx {
  hipStream_t s = nullptr;
  Arena *arena = nullptr;
  bool timing = true;            // per-phase HIP events (none when false)
  uint64_t *h_status = nullptr;  // pinned, 4096 u64
  uint64_t *d_status = nullptr;  // device, 4096 u64
  void sync() { FL_HIP(hipStreamSynchronize(s)); }
  // copy `count` u64 status words from device to host and wait
  void fetch(const void *dev, size_t bytes) {
    FL_HIP(hipMemcpyAsync(h_status, dev, bytes, hipMemcpyDeviceToHost, s));
    sync();
  }
};

// ---------------------------------------------------------------------------
// Validated graph description used by every phase (device pointers).
// ---------------------------------------------------------------------------
// row_ptr/col/w: the arcs out of each vertex (the caller's CSR).  in_*: the
// arcs into each vertex (row v lists the u with an arc u -> v, with its
// weight); the same arrays when the graph is undirected.  Work that moves
// along arcs reads the out-arcs when it pushes from a vertex and the in-arcs
// when it pulls into one; a search for distances TO a set of vertices pushes
// over the in-arcs.
struct Graph {
  uint32_t n;
  uint64_t m;
  const uint64_t *row_ptr;
  const uint32_t *col;
  const uint32_t *w;  // nullptr = unit weights
  uint32_t max_w;
  const uint64_t *in_ptr = nullptr;
  const uint32_t *in_col = nullptr;
  const uint32_t *in_w = nullptr;
  // out-arc a -> its position in the in-arc rows (directed graphs: filled by
  // set_in_arcs; undirected: nullptr, the sketch rounds derive it)
  const uint32_t *out_to_in = nullptr;
};

// Per-slot queue counters, which every wave of a round increments, sit one
// per 128-byte line (CNT_PAD u32 apart): packed together, the ~100 counters
// of a weighted graph share a few lines and every append of the round queues
// on them.
constexpr uint32_t CNT_PAD = 32;
// host copy of `count` padded counters (dense in `host`); waits.  The slot
// ring has at most MAX_W + 1 counters, so the padded array is at most 32 KB.
inline void fetch_padded(Ctx &c, uint32_t *host, const uint32_t *dev, uint32_t count) {
  std::vector<uint32_t> tmp((size_t)count * CNT_PAD);
  FL_HIP(hipMemcpyAsync(tmp.data(), dev, tmp.size() * 4, hipMemcpyDeviceToHost, c.s));
  c.sync();
  for (uint32_t i = 0; i < count; ++i) host[i] = tmp[(size_t)i * CNT_PAD];
}

// fill / utility launches (fl_graph.hip)
void fill_u32(Ctx &c, uint32_t *p, uint64_t n, uint32_t v);
void fill_u64(Ctx &c, uint64_t *p, uint64_t n, uint64_t v);
void fill_u8(Ctx &c, uint8_t *p, uint64_t n, uint8_t v);
void fill_f64(Ctx &c, double *p, uint64_t n, double v);
int validate_graph(Ctx &c, const fl_problem *p, bool directed, uint32_t *max_w_out, uint32_t *max_cost_out);
// Sets g's in-arc view: the out-arc arrays themselves (undirected), or their
// transpose built in the arena (directed; g must be validated).
void set_in_arcs(Ctx &c, Graph &g, bool directed);
size_t transpose_bytes(uint32_t n, uint64_t m, bool weighted);
// validates G graphs (one launch each, one readback); rc/max_w/max_cost per graph
void validate_graphs(Ctx &c, const fl_problem *const *ps, uint32_t G, bool directed, std::vector<int> &rc,
                     std::vector<uint32_t> &max_w, std::vector<uint32_t> &max_cost);
// per-graph sums (or, for the last field with max_last, maxima) of striped
// device counters laid out as [(g * nf + f) * stripes + s]
std::vector<uint64_t> read_seg_ctr(Ctx &c, const uint64_t *d, uint32_t G, uint32_t nf, uint32_t stripes,
                                   bool max_last = false);
// exclusive scan of u32 counts into u64 offsets (out has n+1 entries); sums:
// scan_sums_count(n) words of scratch, or nullptr to take them from the arena
void scan_u32_to_u64(Ctx &c, const uint32_t *in, uint64_t *out, uint32_t n, uint64_t *sums = nullptr);
size_t scan_sums_count(uint32_t n);
// per graph: sum_v cnt[v] * deg(v) and sum_v cnt[v]
void ads_totals(Ctx &c, const Graph &g, const uint32_t *gid, uint32_t G, const uint32_t *cnt,
                std::vector<uint64_t> &relax_alg, std::vector<uint64_t> &entries);

// Multi-source Bellman-Ford with packed 64-bit labels (value << 32 | tie).
// Labels move along arcs by adding w << 32.  `labels` holds the initial
// labels (INF64 = none) and receives the fixed point; `seeds` lists the
// vertices whose label was lowered since the last call (the first frontier).
struct SsspWork {
  uint32_t *front[2];
  uint32_t *flag;  // n: iteration stamp of the last frontier a vertex joined
  uint64_t *heavy; // pieces of the long rows of the current iteration
  uint64_t *ctr;   // device counters: u32 [0], [1] frontier sizes, [2] long rows
  uint32_t stamp = 0;  // stamps grow across calls on this workspace
};
void sssp_alloc(Ctx &c, SsspWork &wk, uint32_t n, uint64_t m);
uint32_t sssp_run(Ctx &c, const Graph &g, uint64_t *labels, const uint32_t *seeds, uint32_t nseeds,
                  SsspWork &wk, uint64_t cap_value);

}  // namespace fl
