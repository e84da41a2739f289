// fl_ads.hip -- bottom-k all-distances sketches (ADS, Sec. 3.3) by rounds of
// edge relaxation on the GPU.
//
// Schedule.  Round D settles every sketch entry at distance exactly D (integer
// weights >= 1).  A candidate (r, D) reaches u from an in-neighbour v over an
// arc v -> u of weight w only if v inserted r in round D - w, so all entries at smaller
// distances are final when round D runs: sketches grow append-only, already in
// (distance, id) order, and no entry is ever evicted (the CleanUp of Alg. 2 is
// never needed).  With unit weights this is the superstep order of Alg. 2.
// Entries move along arcs, so on a directed graph the sketch of u holds the
// vertices that reach u, at d(v, u) (an undirected graph is read as both arcs).
//
// Work items.  A vertex with at most TASK_ARCS arcs (TASK_ARCS_SPARSE in
// rounds run from worklists) is one task; a larger one is split into tasks of
// that many arcs.  Each task (one wave64) streams the
// entries its neighbours inserted at distance D - w (pull), drops those whose
// rank is not below T_u (the k-th smallest rank of u's sketch so far: k
// entries that all come first have a smaller rank) and those already in u's
// bottom-k set, and prunes the rest.  A split vertex's tasks leave their kept
// sets in scratch; a merge wave prunes their union (the prune is associative
// and idempotent, so the split does not change the result).
//
// Level records and arc planes.  The level a vertex commits at distance D is
// described in slot D % NS of its record ring (start, count and its two
// smallest ranks), so a level of one or two entries needs no further read and
// a level whose smallest rank fails the reader's threshold is skipped whole.
// In rounds run from worklists, the committing vertex also sets, for each arc
// it marks, the bit of the arc's position in the head's in-arc row in the
// bit plane of the round the level reaches the head; a task then reads only
// the arcs whose bits are set instead of every in-arc.
//
// Level prune.  A candidate of level D is accepted iff fewer than k ranks
// below its own belong to entries that come first: the sketch so far, or
// level-D candidates with a smaller vertex id (ties in distance go by id).
// Candidates are counting-sorted into id buckets; buckets are walked in id
// order, filtered in parallel against the running k-th smallest rank, and
// the survivors of a bucket are decided 64 at a time by one parallel count
// (set elements below + earlier candidates of the chunk below < k).
// Levels are stored in increasing rank order while the rounds run (a
// neighbour reads one only up to its threshold); the rows that need the
// canonical order (those with a HIP-threshold row) also receive each level in
// id order, in their threshold row, at commit.  A last pass moves that order
// into the sketch row and computes the HIP thresholds T_j (k-th smallest
// rank before entry j) in its place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "fl_ads.h"
#include "fl_common.h"

namespace fl {

constexpr int TASK_WPB = 1;         // waves per block of the round kernels: a block's LDS is
                                    // freed when its own task ends (task lengths vary widely)
// Survivor buffer of a level (ids per wave): ADS_SB for k <= 64, twice that
// for k <= 128.  A level accepts about k (1 + ln(N / k)) of its N candidates
// (453 for k = 32 and N = 2^24), so k <= 32 starts with half the buffer: the
// round kernel then fits 5 waves per SIMD instead of 4.  A level that
// overflows it anyway restarts the build with the full buffer.
constexpr uint32_t ADS_SB = 1024;
static_assert((ADS_SB & (ADS_SB - 1)) == 0, "wave_sort_lds pads to a power of two inside the buffer");
inline uint32_t ads_full_sb(uint32_t k) { return k > 64 ? 2 * ADS_SB : ADS_SB; }
constexpr uint32_t TASK_ARCS = 1024;  // arcs per task of a split vertex in dense rounds (the fewest)
// Sparse rounds (worklists) cut only longer rows: there a hub is active in
// most rounds but few of its arcs bring candidates, and every split costs a
// merge that prunes the tasks' kept sets again.  Results do not depend on the
// cut (a candidate accepted over all arcs is accepted within its piece, and
// the merge prunes the union exactly).
constexpr uint32_t TASK_ARCS_SPARSE = 2048;
static_assert(TASK_ARCS_SPARSE >= TASK_ARCS, "scratch slots are sized for TASK_ARCS");
// With arc bit planes a task reads only the arcs that carry a level, so its
// cost follows those, not its length: rows are cut far less often.
constexpr uint32_t TASK_ARCS_FLAGGED = 8192;
// Rounds read flagged arcs only from FLAG_FROM_RINGS times the slot ring
// (max weight + 1) on, and commits set plane bits from a ring earlier (the
// levels those rounds read).  With one task per wave, scanning every in-arc
// cost less while most vertices were active (1 ring); with two small tasks
// per wave the planes pay from the first round (0): a task reads only the
// arcs that carry a level, and rows split at TASK_ARCS_FLAGGED from the start.
constexpr uint32_t FLAG_FROM_RINGS = 0;
static_assert(TASK_ARCS_FLAGGED >= TASK_ARCS, "scratch slots are sized for TASK_ARCS");
constexpr uint32_t NBKT = 64;       // id buckets of the level prune (one per lane)
constexpr uint32_t LONG_LIST = 64;  // entry lists at least this long are streamed one arc at a time

// Statistics counters of the sketch rounds, cumulative over a build: one
// 128-byte line per stripe holds every field, and a block adds into stripe
// blockIdx.x % CTR_STRIPES (a field striped over consecutive words would put
// ~16 blocks on each line).
constexpr uint32_t CTR_STRIPES = 256, CTR_FIELDS = 16;
enum CtrField : uint32_t {
  CF_EXAMINED = 0,  // relaxations executed
  CF_COMMITS,       // levels committed (vertices that changed)
  CF_SURVIVORS,     // candidates kept after the offer filters
  CF_PRUNES,        // level prunes
  CF_SCANNED,       // arcs scanned (dbg)
  CF_MATCHED,       // level records matched (dbg)
  CF_MARK_ARCS,     // arcs examined for marking (dbg)
  CF_MARKED,        // heads that passed the marking filter (dbg)
  CF_COUNT
};
struct AdsArgs {
  uint32_t n, k, cap, W, NS, FW;
  const uint32_t *gid;  // graph of each vertex (nullptr: one graph)
  const SegInfo *seg;   // per-graph rank keys, base, bucket shift
  // entries travel along arcs: a vertex gathers over its in-arcs and, when
  // its sketch changes, marks the heads of its out-arcs (one CSR twice when
  // the graph is undirected)
  const uint64_t *row_ptr;  // in-arcs
  const uint32_t *col;
  const uint32_t *w;
  const uint64_t *out_ptr;  // out-arcs
  const uint32_t *out_col;
  const uint32_t *out_w;
  uint32_t *sk_rank;
  uint32_t *sk_dist;
  uint32_t *bk;
  uint32_t *cnt;
  uint4 *lvl;          // [NS * n] level records, slot (D % NS) of each vertex
  uint32_t *flags;
  uint32_t *wl;
  uint32_t *wl_cnt;
  // arc bit planes of the rounds run from worklists (nullptr: scan every in-arc)
  uint32_t *plane;            // [NS * pw] bit of in-arc position p set in plane D % NS: a level reaches it in round D
  uint64_t pw;                // words per plane
  uint32_t flag_from;         // first round whose tasks read only flagged arcs
  uint32_t plane_from;        // first round whose commits set plane bits (flag_from - max weight)
  const uint32_t *out_to_in;  // [m] out-arc -> in-arc position
  uint32_t *kept;      // [slots * sb] kept ids of split tasks
  uint32_t sb;         // survivor buffer of the build (the round kernels' template argument)
  uint32_t *kept_cnt;  // [slots]
  uint64_t *ctr;       // [CTR_STRIPES * CTR_FIELDS] cumulative counters, see CtrField
  uint32_t dbg;
  uint32_t *status;    // [0] capacity overflow, [1] survivor-buffer overflow
  uint32_t *thr;             // [rows * cap] threshold rows: canonical-order ranks until the last pass
  const uint32_t *thr_idx;   // [n] threshold row of each vertex (INF32 = none); nullptr = row u
};

__device__ inline uint32_t thr_row(const AdsArgs &P, uint32_t u) {
  return P.thr ? (P.thr_idx ? P.thr_idx[u] : u) : INF32;
}

__device__ inline void ctr_add(const AdsArgs &P, CtrField f, uint64_t v) {
  atomicAdd((unsigned long long *)&P.ctr[(blockIdx.x % CTR_STRIPES) * CTR_FIELDS + f], (unsigned long long)v);
}

// The level a vertex committed at distance D stays in slot D % NS until the
// level at D + NS reuses it: {D, its smallest rank, its second smallest rank
// (INF32 for a single entry), start | count << 16}.  A level is stored in
// increasing rank order, so a reader whose threshold is at most the smallest
// rank skips it whole, and a level of one or two entries is read from the
// record alone.
__device__ inline uint4 level_record(uint32_t D, uint32_t r0, uint32_t r1, uint32_t start, uint32_t count) {
  return make_uint4(D, r0, r1, start | (count << 16));
}

// Append y to the worklist of slot s once (flag bit per (vertex, slot)).
// Lanes with want=false do nothing.
template <bool UNITW>
__device__ inline void mark_targets(const AdsArgs &P, bool want, uint32_t y, uint32_t s) {
  bool add = false;
  if (want) {
    uint32_t *word = &P.flags[(size_t)y * P.FW + (s >> 5)];
    const uint32_t bit = 1u << (s & 31);
    if (!(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit))
      add = !(atomicOr(word, bit) & bit);
  }
  if (UNITW) {
    // every lane's slot is D + 1: one atomic per wave
    wave_push(P.wl + (size_t)s * P.n, &P.wl_cnt[s * CNT_PAD], add, y);
  } else if (add) {
    // the lanes' slots are mostly distinct (about 47 of 64 for weights
    // 1..100): one atomic per lane costs less than grouping them by slot
    const uint32_t pos = atomicAdd(&P.wl_cnt[s * CNT_PAD], 1u);
    P.wl[(size_t)s * P.n + pos] = y;
  }
}

// u committed a level at distance D: queue each head y of an arc u -> y for
// round D + w, and set the arc's bit in that round's plane.  Several waves
// can share a long row: wave `part` of `parts` takes every parts-th group of
// 64 arcs.
template <bool UNITW>
__device__ inline void mark_neighbours(const AdsArgs &P, uint32_t u, uint32_t D, uint32_t part = 0,
                                       uint32_t parts = 1) {
  const int lane = lane_id();
  const uint64_t a0 = P.out_ptr[u], a1 = P.out_ptr[u + 1];
  for (uint64_t b = a0 + (uint64_t)part * WAVE; b < a1; b += (uint64_t)parts * WAVE) {
    const uint64_t a = b + lane;
    bool want = a < a1;
    uint32_t y = 0, s = 0;
    if (want) {
      y = P.out_col[a];
      const uint32_t wv = UNITW ? 1u : P.out_w[a];
      s = (D + wv) % P.NS;
      if (P.plane && D >= P.plane_from) {
        const uint32_t p = P.out_to_in[a];
        atomicOr(&P.plane[(size_t)s * P.pw + (p >> 5)], 1u << (p & 31));
      }
    }
    if (P.dbg) {
      const uint64_t wm = __ballot(want);
      if (lane == 0) {
        ctr_add(P, CF_MARK_ARCS, a1 - b < WAVE ? a1 - b : WAVE);
        ctr_add(P, CF_MARKED, __popcll(wm));
      }
    }
    mark_targets<UNITW>(P, want, y, s);
  }
}

// Round 0: every vertex holds (r(v), 0).  One wave per vertex.
template <bool UNITW>
__global__ __launch_bounds__(256) void k_ads_init(AdsArgs P, int mark) {
  const int lane = lane_id();
  const uint64_t u64 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (u64 >= P.n) return;
  const uint32_t u = (uint32_t)u64;
  const uint32_t r = rank_of(u, rank_map(P.seg[seg_of(P.gid, u)]));
  if (lane == 0) {
    P.sk_rank[(size_t)u * P.cap] = r;
    P.sk_dist[(size_t)u * P.cap] = 0;
    const uint32_t tr = thr_row(P, u);
    if (tr != INF32) P.thr[(size_t)tr * P.cap] = r;
    P.bk[(size_t)u * P.k] = r;
    P.cnt[u] = 1;
    P.lvl[u] = level_record(0, r, INF32, 0, 1);  // slot 0
  }
  if (mark) mark_neighbours<UNITW>(P, u, 0);
}

// ---------------------------------------------------------------------------
// sorting helpers
// ---------------------------------------------------------------------------
// Sort s[0..n) ascending in LDS (bitonic over the next power of two; the
// caller guarantees that many slots).
__device__ inline void wave_sort_lds(uint32_t *s, uint32_t n) {
  const int lane = lane_id();
  uint32_t p2 = 2;
  while (p2 < n) p2 <<= 1;
  for (uint32_t i = n + lane; i < p2; i += WAVE) s[i] = INF32;
  wave_lds_sync();
  for (uint32_t k2 = 2; k2 <= p2; k2 <<= 1) {
    for (uint32_t j = k2 >> 1; j > 0; j >>= 1) {
      for (uint32_t i = lane; i < p2; i += WAVE) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint32_t a = s[i], b = s[ixj];
          if ((a > b) == ((i & k2) == 0)) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

// Sort one value per lane ascending across the wave (bitonic network).
__device__ inline uint32_t wave_sort_reg(uint32_t x) {
  const int lane = lane_id();
#pragma unroll
  for (int k2 = 2; k2 <= WAVE; k2 <<= 1) {
#pragma unroll
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      const uint32_t y = __shfl_xor(x, j, WAVE);
      const bool keep_min = ((lane & k2) == 0) == ((lane & j) == 0);
      x = keep_min ? (x < y ? x : y) : (x > y ? x : y);
    }
  }
  return x;
}

// Values of lanes 0..n-1 (n <= 64; lanes from n on hold INF32) sorted
// ascending onto lanes 0..n-1, INF32 above.  Each lane counts the staged
// values that come before its own (smaller, or equal on a lower lane), four
// per LDS read, and writes its value there: for a few values this is cheaper
// than the 21 exchange steps of the bitonic network.  s_r: 64 words, 16-byte
// aligned, free on entry and on return.
constexpr uint32_t COUNT_SORT_MAX = 16;
__device__ inline uint32_t wave_sort_few(uint32_t x, uint32_t n, uint32_t *s_r) {
  const uint32_t lane = (uint32_t)lane_id();
  s_r[lane] = x;
  wave_lds_sync();
  uint32_t pos = 0;
  for (uint32_t j4 = 0; j4 < n; j4 += 4) {
    const uint4 v = *reinterpret_cast<const uint4 *>(&s_r[j4]);
    pos += (v.x < x || (v.x == x && j4 + 0 < lane)) ? 1u : 0u;
    pos += (v.y < x || (v.y == x && j4 + 1 < lane)) ? 1u : 0u;
    pos += (v.z < x || (v.z == x && j4 + 2 < lane)) ? 1u : 0u;
    pos += (v.w < x || (v.w == x && j4 + 3 < lane)) ? 1u : 0u;
  }
  wave_lds_sync();
  if (lane < n) s_r[pos] = x;
  wave_lds_sync();
  const uint32_t y = lane < n ? s_r[lane] : INF32;
  wave_lds_sync();
  return y;
}

// Merge of a bitonic sequence held one value per lane into ascending
// (desc = false) or descending order.
__device__ inline uint32_t wave_bitonic_merge(uint32_t x, bool desc) {
  const int lane = lane_id();
#pragma unroll
  for (int j = 32; j >= 1; j >>= 1) {
    const uint32_t y = __shfl_xor(x, j, WAVE);
    const bool lo = ((lane & j) == 0) != desc;
    x = lo ? (x < y ? x : y) : (x > y ? x : y);
  }
  return x;
}

// Two ascending sequences a and b, one value per lane: lo receives the 64
// smallest of both, hi the 64 largest, each ascending (the first step of a
// bitonic merge splits them into two bitonic halves).
__device__ inline void wave_merge2(uint32_t a, uint32_t b, uint32_t &lo, uint32_t &hi) {
  const uint32_t br = __shfl(b, WAVE - 1 - lane_id(), WAVE);
  lo = wave_bitonic_merge(a < br ? a : br, false);
  hi = wave_bitonic_merge(a < br ? br : a, false);
}

// The running bottom-k set of a level: ascending, element i in register
// i / 64 at lane i % 64, INF32 above its size.  One register holds k <= 64,
// two hold k <= 128.
template <int KR>
struct KSet {
  uint32_t v[KR];
};

// element i of the set (i per lane, below 64 KR)
template <int KR>
__device__ inline uint32_t kset_at(const KSet<KR> &s, uint32_t i) {
  if (KR == 1) return __shfl(s.v[0], (int)i, WAVE);
  const uint32_t a = __shfl(s.v[0], (int)(i & 63u), WAVE);
  const uint32_t b = __shfl(s.v[KR - 1], (int)(i & 63u), WAVE);
  return i < 64u ? a : b;
}

// number of set elements below the wave-uniform rank rj
template <int KR>
__device__ inline uint32_t kset_ballot_below(const KSet<KR> &s, uint32_t rj) {
  uint32_t c = (uint32_t)__popcll(__ballot(s.v[0] < rj));
  if (KR == 2) c += (uint32_t)__popcll(__ballot(s.v[KR - 1] < rj));
  return c;
}

// insert the wave-uniform rank rj at position below, keeping k elements
template <int KR>
__device__ inline void kset_insert(KSet<KR> &s, uint32_t rj, uint32_t below, uint32_t k) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t up0 = __shfl_up(s.v[0], 1, WAVE);
  if (KR == 2) {
    const uint32_t last0 = __shfl(s.v[0], WAVE - 1, WAVE);
    uint32_t up1 = __shfl_up(s.v[KR - 1], 1, WAVE);
    if (lane == 0) up1 = last0;
    const uint32_t e1 = 64u + lane;
    if (e1 > below && e1 < k) s.v[KR - 1] = up1;
    if (e1 == below) s.v[KR - 1] = rj;
  }
  if (lane > below && lane < k) s.v[0] = up0;
  if (lane == below) s.v[0] = rj;
}

// the set becomes the k smallest of itself and the ascending chunk x
// (INF32-padded)
template <int KR>
__device__ inline void kset_merge(KSet<KR> &s, uint32_t x, uint32_t k) {
  const uint32_t lane = (uint32_t)lane_id();
  if (KR == 1) {
    const uint32_t y = __shfl(x, WAVE - 1 - (int)lane, WAVE);
    uint32_t mm = s.v[0] < y ? s.v[0] : y;  // bitonic, holds the 64 smallest of both
    mm = wave_bitonic_merge(mm, false);
    s.v[0] = lane < k ? mm : INF32;
  } else {
    // the 64 smallest of everything lie in the lower half and the chunk; the
    // next 64 in what is left of those and the upper half
    uint32_t lo1, hi1, lo2, hi2;
    wave_merge2(s.v[0], x, lo1, hi1);
    wave_merge2(hi1, s.v[KR - 1], lo2, hi2);
    s.v[0] = lane < k ? lo1 : INF32;
    s.v[KR - 1] = 64u + lane < k ? lo2 : INF32;
  }
}

// number of values below r in a set held one value per lane, ascending, with
// INF32 above its size (per-lane r; every lane runs the shuffles)
__device__ inline uint32_t set_count_below(uint32_t setv, uint32_t r) {
  uint32_t q = 0;
#pragma unroll
  for (uint32_t s = 32; s >= 1; s >>= 1) {
    const uint32_t val = __shfl(setv, (int)(q + s - 1), WAVE);
    if (val < r) q += s;
  }
  const uint32_t atq = __shfl(setv, (int)q, WAVE);
  if (atq < r) ++q;  // all 64 values below r
  return q;
}

// number of elements of the set below r (per-lane r)
template <int KR>
__device__ inline uint32_t kset_below(const KSet<KR> &s, uint32_t r) {
  const uint32_t q = set_count_below(s.v[0], r);
  if (KR == 1) return q;
  const uint32_t q2 = set_count_below(s.v[KR - 1], r);
  return q == 64u ? 64u + q2 : q;
}

// One chunk of candidates, one id per lane in ascending lane order (INF32 =
// empty slot at the end); duplicates are adjacent; `prev` is the last id of
// the previous chunk of this level.  Candidate i is accepted iff
//   #(running set below r_i) + #(earlier distinct candidates of the chunk below r_i) < k.
// The running set becomes the k smallest ranks of itself and the chunk.
// Returns the mask of accepted lanes.
template <int KR>
__device__ inline uint64_t chunk_accept(uint32_t id, uint32_t k, const RankMap &rm, KSet<KR> &set,
                                        uint32_t &nset, uint32_t &prev, uint32_t *s_r) {
  const int lane = lane_id();
  uint32_t left = __shfl_up(id, 1, WAVE);
  if (lane == 0) left = prev;
  bool valid = id != INF32 && id != left;
  const uint32_t r = valid ? rank_of(id, rm) : INF32;
  const uint32_t q = kset_below(set, r);
  // a candidate already in the set (same vertex at a shorter distance) is
  // not new; one that dropped out of the set is rejected by the count
  const uint32_t atq = kset_at(set, q < 64u * KR - 1u ? q : 64u * KR - 1u);
  if (q < nset && atq == r) valid = false;
  const uint64_t vm = __ballot(valid);
  // earlier candidates of the chunk with a smaller rank: ranks staged in LDS,
  // read four at a time by every lane from the same address (broadcast)
  s_r[lane] = valid ? r : INF32;
  wave_lds_sync();
  const int top = vm ? 64 - __clzll(vm) : 0;  // lanes above the last valid one are empty
  uint32_t cp = 0;
  for (int j4 = 0; j4 < top; j4 += 4) {
    const uint4 v = *reinterpret_cast<const uint4 *>(&s_r[j4]);
    cp += (j4 + 0 < lane && v.x < r) ? 1u : 0u;
    cp += (j4 + 1 < lane && v.y < r) ? 1u : 0u;
    cp += (j4 + 2 < lane && v.z < r) ? 1u : 0u;
    cp += (j4 + 3 < lane && v.w < r) ? 1u : 0u;
  }
  wave_lds_sync();
  const bool acc = valid && q + cp < k;
  const uint64_t am = __ballot(acc);
  // the running set becomes the k smallest of (set, accepted ranks); rejected
  // candidates have k smaller ranks before them and never enter it
  const uint32_t na = (uint32_t)__popcll(am);
  if (na <= 8) {
    uint64_t it2 = am;
    while (it2) {
      const int j = __ffsll((long long)it2) - 1;
      it2 &= it2 - 1;
      const uint32_t rj = __shfl(r, j, WAVE);
      kset_insert(set, rj, kset_ballot_below(set, rj), k);
    }
  } else {
    kset_merge(set, wave_sort_reg(acc ? r : INF32), k);
  }
  const uint32_t tot = nset + na;
  nset = tot < k ? tot : k;
  const uint64_t real = __ballot(id != INF32);
  if (real) prev = __shfl(id, 63 - __clzll(real), WAVE);
  return am;
}

// Prune of one distance level.  s_id[0..ns) holds candidate ids (unsorted,
// duplicates allowed); set/nset the running set.  Accepted ids end in
// s_tmp[0..m) in increasing id order; returns m.  s_id is clobbered.
// s_cnt holds (2 + KR) WAVE words: [0, WAVE) bucket offsets, then the
// pending chunk; [WAVE, (1 + KR) WAVE) belongs to the caller; the last WAVE
// hold chunk ranks.
// With tbk, lane b of *tbk receives a rank bound for id bucket b: the running
// k-th smallest rank when the bucket was reached, which no later candidate of
// that bucket can beat.
template <int KR>
__device__ inline uint32_t prune_level(uint32_t *s_id, uint32_t *s_tmp, uint32_t *s_cnt, uint32_t ns,
                                       uint32_t k, const RankMap &rm, KSet<KR> &set, uint32_t &nset,
                                       uint32_t *tbk = nullptr) {
  const int lane = lane_id();
  uint32_t *s_pend = s_cnt;
  uint32_t *s_r = s_cnt + (1 + KR) * WAVE;
  uint32_t m = 0, prev = INF32;
  if (ns <= (uint32_t)WAVE && !tbk) {
    uint32_t x = (uint32_t)lane < ns ? s_id[lane] : INF32;
    x = ns <= COUNT_SORT_MAX ? wave_sort_few(x, ns, s_r) : wave_sort_reg(x);
    const uint64_t am = chunk_accept(x, k, rm, set, nset, prev, s_r);
    if ((am >> lane) & 1) s_tmp[lanes_below(am)] = x;
    wave_lds_sync();
    return (uint32_t)__popcll(am);
  }
  // counting sort by id bucket (bucket order is id order)
  s_cnt[lane] = 0;
  wave_lds_sync();
  for (uint32_t i = lane; i < ns; i += WAVE) atomicAdd(&s_cnt[bucket_of(s_id[i], rm)], 1u);
  wave_lds_sync();
  const uint32_t bc = s_cnt[lane];
  const uint32_t bstart = wave_scan_incl(bc) - bc;
  wave_lds_sync();
  s_cnt[lane] = bstart;
  wave_lds_sync();
  for (uint32_t i = lane; i < ns; i += WAVE) {
    const uint32_t id = s_id[i];
    s_tmp[atomicAdd(&s_cnt[bucket_of(id, rm)], 1u)] = id;
  }
  wave_lds_sync();
  // Buckets are walked in id order.  The survivors of consecutive buckets are
  // gathered in one pending chunk of at most WAVE ids and decided together;
  // accepted ids are written back to s_tmp[m..), which never reaches a bucket
  // not yet read (accepted ones are a subset of the buckets already read).
  uint64_t nonempty = __ballot(bc != 0);
  uint32_t tb = INF32;
  int done_b = -1;
  uint32_t npend = 0;
  auto flush = [&]() {
    uint32_t x = (uint32_t)lane < npend ? s_pend[lane] : INF32;
    x = npend <= COUNT_SORT_MAX ? wave_sort_few(x, npend, s_r) : wave_sort_reg(x);
    const uint64_t am = chunk_accept(x, k, rm, set, nset, prev, s_r);
    if ((am >> lane) & 1) s_tmp[m + lanes_below(am)] = x;
    m += (uint32_t)__popcll(am);
    npend = 0;
    wave_lds_sync();
  };
  // keep the ids of bucket [sb, sb + cb) whose rank beats the running
  // threshold, compacted in place; returns their number
  auto filter = [&](uint32_t sb, uint32_t cb) -> uint32_t {
    const bool open = nset < k;
    const uint32_t Trun = open ? INF32 : kset_at(set, k - 1);
    uint32_t np = 0;
    for (uint32_t j0 = 0; j0 < cb; j0 += WAVE) {
      const uint32_t j = j0 + lane;
      uint32_t id = INF32;
      bool pass = false;
      if (j < cb) {
        id = s_tmp[sb + j];
        pass = open || rank_of(id, rm) < Trun;
      }
      const uint64_t pm = __ballot(pass);
      if (pass) s_tmp[sb + np + lanes_below(pm)] = id;
      np += (uint32_t)__popcll(pm);
    }
    wave_lds_sync();
    return np;
  };
  while (nonempty) {
    const int b = __ffsll((long long)nonempty) - 1;
    nonempty &= nonempty - 1;
    const uint32_t cb = __shfl(bc, b, WAVE);
    const uint32_t sb = __shfl(bstart, b, WAVE);
    // the running threshold now bounds every bucket up to b
    const uint32_t Tnow = nset < k ? INF32 : kset_at(set, k - 1);
    if (lane > done_b && lane <= b) tb = Tnow;
    done_b = b;
    uint32_t np = filter(sb, cb);
    if (np == 0) continue;
    if (npend + np > (uint32_t)WAVE) {
      flush();
      // every earlier candidate is decided: the threshold is exact for bucket b
      const uint32_t T2 = nset < k ? INF32 : kset_at(set, k - 1);
      if (lane == b) tb = T2;
      np = filter(sb, np);
      if (np == 0) continue;
    }
    if (np > (uint32_t)WAVE) {
      // many survivors in one bucket: sort them in s_id (free now), then chunks in order
      for (uint32_t i = lane; i < np; i += WAVE) s_id[i] = s_tmp[sb + i];
      wave_sort_lds(s_id, np);
      for (uint32_t c0 = 0; c0 < np; c0 += WAVE) {
        const uint32_t x = c0 + lane < np ? s_id[c0 + lane] : INF32;
        const uint64_t am = chunk_accept(x, k, rm, set, nset, prev, s_r);
        if ((am >> lane) & 1) s_tmp[m + lanes_below(am)] = x;
        m += (uint32_t)__popcll(am);
        wave_lds_sync();
      }
      continue;
    }
    if ((uint32_t)lane < np) s_pend[npend + lane] = s_tmp[sb + lane];
    npend += np;
    wave_lds_sync();
  }
  if (npend) flush();
  if (tbk) {
    const uint32_t Tend = nset < k ? INF32 : kset_at(set, k - 1);
    if (lane > done_b) tb = Tend;
    *tbk = tb;
  }
  return m;
}

// ---------------------------------------------------------------------------
// per-wave level state: candidate intake with filtering and buffering
// ---------------------------------------------------------------------------
template <int KR>
struct Level {
  KSet<KR> set0;         // u's bottom-k set at the start of the level
  uint32_t nset0;
  uint32_t T0;           // its k-th smallest rank (INF32 while fewer than k)
  bool full0;
  uint32_t cu;           // entries of u so far
  uint32_t ns;           // buffered candidates
  uint32_t tb;           // lane b < NBKT: rank bound for candidates of id bucket b
  RankMap rm;            // ranks and id buckets of u's graph
  bool overflow;
  uint32_t nsurv, nprune;  // statistics
  uint32_t nmatch;         // level records found (per lane; with dbg only)
};

template <int KR>
__device__ inline void level_init(const AdsArgs &P, uint32_t u, Level<KR> &L, uint32_t *s_cnt) {
  const int lane = lane_id();
  const uint32_t k = P.k;
  L.rm = rank_map(P.seg[seg_of(P.gid, u)]);
  L.cu = P.cnt[u];
  L.nset0 = L.cu < k ? L.cu : k;
#pragma unroll
  for (int g = 0; g < KR; ++g) {
    const uint32_t e = (uint32_t)(64 * g + lane);
    L.set0.v[g] = e < L.nset0 ? P.bk[(size_t)u * k + e] : INF32;
    s_cnt[WAVE + e] = L.set0.v[g];
  }
  wave_lds_sync();
  L.full0 = L.nset0 == k;
  L.T0 = L.full0 ? kset_at(L.set0, k - 1) : INF32;
  L.ns = 0;
  L.tb = L.T0;
  L.overflow = false;
  L.nsurv = L.nprune = L.nmatch = 0;
}

// One candidate per lane (valid, rank r, id if known): keep it if its rank is
// below T0 and it is not already in the set; buffer kept ids, shrinking the
// buffer by a prune against the set when full.
template <int KR, uint32_t SB>
__device__ inline void level_offer(const AdsArgs &P, Level<KR> &L, bool valid, uint32_t r, bool have_id, uint32_t id,
                                   uint32_t *s_id, uint32_t *s_tmp, uint32_t *s_cnt) {
  const uint32_t *s_set0 = s_cnt + WAVE;  // LDS copy of the set at the level start
  const int lane = lane_id();
  bool pass = valid && (!L.full0 || r < L.T0);
  if (!__ballot(pass)) return;
  if (pass) {
    // already in the set (same vertex at a shorter distance)?
    uint32_t lo = 0, hi = L.nset0;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_set0[mid] < r) lo = mid + 1;
      else hi = mid;
    }
    if (lo < L.nset0 && s_set0[lo] == r) pass = false;
  }
  // bucket bound from the last prune: all candidates of earlier id buckets
  // come first, and k of them (or of the set) already rank below it
  const uint32_t cid = pass ? (have_id ? id : id_of(r, L.rm)) : L.rm.base;
  const uint32_t bnd = __shfl(L.tb, (int)bucket_of(cid, L.rm), WAVE);
  if (pass && r >= bnd) pass = false;
  uint64_t msk = __ballot(pass);
  if (!msk) return;
  uint32_t np = (uint32_t)__popcll(msk);
  if (L.ns + np > SB) {
    KSet<KR> tv = L.set0;
    uint32_t tn = L.nset0;
    ++L.nprune;
    L.ns = prune_level(s_id, s_tmp, s_cnt, L.ns, P.k, L.rm, tv, tn, &L.tb);
    for (uint32_t i = lane; i < L.ns; i += WAVE) s_id[i] = s_tmp[i];
    wave_lds_sync();
    // the new bounds may reject some of this chunk too
    const uint32_t bnd2 = __shfl(L.tb, (int)bucket_of(cid, L.rm), WAVE);
    if (pass && r >= bnd2) pass = false;
    msk = __ballot(pass);
    np = (uint32_t)__popcll(msk);
    if (L.ns + np > SB) {
      L.overflow = true;
      return;
    }
  }
  if (pass) s_id[L.ns + lanes_below(msk)] = cid;
  L.ns += np;
  L.nsurv += np;
  wave_lds_sync();
}

// One in-arc per lane (arc index a, valid): the level each arc's tail
// committed at distance D - w is offered to u's level D.  Levels of one or
// two entries come from the record; longer ones from the tail's sketch row,
// the whole wave on one list at a time when it is long (a level is stored in
// increasing rank order, so once a rank reaches T0 the rest cannot enter).
template <bool UNITW, int KR, uint32_t SB>
__device__ inline uint64_t gather_batch(const AdsArgs &P, uint32_t D, uint64_t a, bool valid, Level<KR> &L,
                                        uint32_t *s_id, uint32_t *s_tmp, uint32_t *s_cnt) {
  const int lane = lane_id();
  uint64_t examined = 0;
  {
    uint32_t v = 0, st = 0, cn = 0, r0 = INF32, r1 = INF32;
    if (valid) {
      v = P.col[a];
      const uint32_t wv = UNITW ? 1u : P.w[a];
      if (wv <= D) {
        const uint32_t src = D - wv;
        const uint4 rec = P.lvl[(size_t)(src % P.NS) * P.n + v];
        // a level whose smallest rank is not below T0 has nothing for u
        if (P.dbg && rec.x == src) ++L.nmatch;
        if (rec.x == src && (!L.full0 || rec.y < L.T0)) {
          r0 = rec.y;
          r1 = rec.z;
          st = rec.w & 0xFFFFu;
          cn = rec.w >> 16;
        }
      }
    }
    // levels of one or two entries: the ranks are in the record
    {
      const bool one = cn != 0 && cn <= 2;
      const bool two = cn == 2;
      examined += __popcll(__ballot(one)) + __popcll(__ballot(two));
      level_offer<KR, SB>(P, L, one, r0, false, 0, s_id, s_tmp, s_cnt);
      if (__ballot(two) && !L.overflow) level_offer<KR, SB>(P, L, two, r1, false, 0, s_id, s_tmp, s_cnt);
      if (cn <= 2) cn = 0;
    }
    // long lists: one arc at a time, the whole wave on its list, four loads in
    // flight.  A level is stored in increasing rank order, so once a rank
    // reaches T0 the rest of the list cannot enter u's sketch.
    uint64_t lm = __ballot(cn >= LONG_LIST);
    while (lm && !L.overflow) {
      const int j = __ffsll((long long)lm) - 1;
      lm &= lm - 1;
      const uint32_t vj = __shfl(v, j, WAVE);
      const uint32_t stj = __shfl(st, j, WAVE);
      const uint32_t cnj = __shfl(cn, j, WAVE);
      const uint32_t *src = P.sk_rank + (size_t)vj * P.cap + stj;
      for (uint32_t c0 = 0; c0 < cnj && !L.overflow; c0 += 4 * WAVE) {
        const uint32_t i0 = c0 + lane, i1 = i0 + WAVE, i2 = i1 + WAVE, i3 = i2 + WAVE;
        const uint32_t r0 = i0 < cnj ? src[i0] : INF32;
        const uint32_t r1 = i1 < cnj ? src[i1] : INF32;
        const uint32_t r2 = i2 < cnj ? src[i2] : INF32;
        const uint32_t r3 = i3 < cnj ? src[i3] : INF32;
        // entries offered (a block past the stop test is loaded, not counted)
        const uint32_t left = cnj - c0;
        examined += left < WAVE ? left : WAVE;
        level_offer<KR, SB>(P, L, i0 < cnj, r0, false, 0, s_id, s_tmp, s_cnt);
        if (L.full0 && __ballot(i0 < cnj && r0 >= L.T0)) break;
        if (c0 + WAVE < cnj) {
          examined += left - WAVE < WAVE ? left - WAVE : WAVE;
          level_offer<KR, SB>(P, L, i1 < cnj, r1, false, 0, s_id, s_tmp, s_cnt);
        }
        if (L.full0 && __ballot(i1 < cnj && r1 >= L.T0)) break;
        if (c0 + 2 * WAVE < cnj) {
          examined += left - 2 * WAVE < WAVE ? left - 2 * WAVE : WAVE;
          level_offer<KR, SB>(P, L, i2 < cnj, r2, false, 0, s_id, s_tmp, s_cnt);
        }
        if (L.full0 && __ballot(i2 < cnj && r2 >= L.T0)) break;
        if (c0 + 3 * WAVE < cnj) {
          examined += left - 3 * WAVE < WAVE ? left - 3 * WAVE : WAVE;
          level_offer<KR, SB>(P, L, i3 < cnj, r3, false, 0, s_id, s_tmp, s_cnt);
        }
        if (L.full0 && __ballot(i3 < cnj && r3 >= L.T0)) break;
      }
    }
    // short lists: flattened over the group, owner lane found by binary search
    const uint32_t cs = cn < LONG_LIST ? cn : 0u;
    const uint32_t incl = wave_scan_incl(cs);
    const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
    const uint32_t excl = incl - cs;
    examined += total;
    for (uint32_t c0 = 0; c0 < total && !L.overflow; c0 += WAVE) {
      const uint32_t idx = c0 + lane;
      uint32_t pos = 0;  // owner lane: first lane whose inclusive count exceeds idx
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
      level_offer<KR, SB>(P, L, valid, r, false, 0, s_id, s_tmp, s_cnt);
    }
  }
  return examined;
}

// Stream the candidates of arcs [a0, a1) of u for level D (every in-arc is
// looked at: rounds run over the dense vertex list).
template <bool UNITW, int KR, uint32_t SB>
__device__ inline uint64_t gather_arcs(const AdsArgs &P, uint32_t D, uint64_t a0, uint64_t a1, Level<KR> &L,
                                       uint32_t *s_id, uint32_t *s_tmp, uint32_t *s_cnt) {
  const int lane = lane_id();
  uint64_t examined = 0;
  for (uint64_t b = a0; b < a1 && !L.overflow; b += WAVE)
    examined += gather_batch<UNITW, KR, SB>(P, D, b + lane, b + lane < a1, L, s_id, s_tmp, s_cnt);
  return examined;
}

// Rounds run from worklists: a tail that committed a level set the bit of
// each arc it marked, at the arc's position in the in-arc rows, in the plane
// of the round the level reaches the head.  Only those arcs of [a0, a1) are
// read: 64 plane words per step, their set bits compacted over the wave.
template <bool UNITW, int KR, uint32_t SB>
__device__ inline uint64_t gather_flagged(const AdsArgs &P, uint32_t D, uint64_t a0, uint64_t a1, Level<KR> &L,
                                          uint32_t *s_id, uint32_t *s_tmp, uint32_t *s_cnt) {
  const int lane = lane_id();
  const uint32_t *plane = P.plane + (size_t)(D % P.NS) * P.pw;
  const uint64_t w0 = a0 >> 5, w1 = (a1 + 31) >> 5;
  uint64_t examined = 0;
  for (uint64_t wb = w0; wb < w1 && !L.overflow; wb += WAVE) {
    const uint64_t wi = wb + lane;
    uint32_t bits = 0;
    if (wi < w1) {
      bits = plane[wi];
      const uint64_t base = wi << 5;  // arcs [base, base + 32) of this word
      if (base < a0) bits &= ~0u << (uint32_t)(a0 - base);
      if (a1 - base < 32) bits &= (1u << (uint32_t)(a1 - base)) - 1u;
    }
    const uint32_t nb = (uint32_t)__popc(bits);
    const uint32_t incl = wave_scan_incl(nb);
    const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
    for (uint32_t c0 = 0; c0 < total && !L.overflow; c0 += WAVE) {
      const uint32_t idx = c0 + lane;
      uint32_t pos = 0;  // word (lane) holding set bit idx: first lane whose inclusive count exceeds idx
#pragma unroll
      for (uint32_t sh = 32; sh >= 1; sh >>= 1) {
        const uint32_t val = __shfl(incl, (int)(pos + sh - 1), WAVE);
        if (val <= idx) pos += sh;
      }
      const bool valid = idx < total;
      const uint32_t src = valid ? pos : 0u;
      uint32_t x = __shfl(bits, (int)src, WAVE);
      uint32_t kth = idx - (__shfl(incl, (int)src, WAVE) - (uint32_t)__popc(x));
      uint32_t bit = 0;  // position of the kth set bit of x
#pragma unroll
      for (uint32_t sh = 16; sh >= 1; sh >>= 1) {
        const uint32_t cnt = (uint32_t)__popc(x & ((1u << sh) - 1u));
        if (kth >= cnt) {
          kth -= cnt;
          x >>= sh;
          bit += sh;
        }
      }
      const uint64_t a = ((wb + src) << 5) + bit;
      examined += gather_batch<UNITW, KR, SB>(P, D, a, valid, L, s_id, s_tmp, s_cnt);
    }
  }
  return examined;
}

// Final prune of u's level-D candidates and the append of the accepted ones.
template <bool UNITW, int KR>
__device__ inline bool level_commit(const AdsArgs &P, uint32_t u, uint32_t D, Level<KR> &L, int mark, uint32_t *s_id,
                                    uint32_t *s_tmp, uint32_t *s_cnt) {
  const int lane = lane_id();
  if (L.ns == 0) return false;
  KSet<KR> set = L.set0;
  uint32_t nset = L.nset0;
  const uint32_t m = prune_level(s_id, s_tmp, s_cnt, L.ns, P.k, L.rm, set, nset);
  if (m == 0) return false;
  const uint32_t cu = L.cu;
  if (cu + m > P.cap) {
    if (lane == 0) atomicOr(&P.status[0], 1u);
    return false;
  }
  // The level is stored in increasing rank order, so that a neighbour reads
  // it only up to its own threshold.  A row with a threshold row also gets the
  // level in id order (the order of s_tmp) there, for the last pass.
  const uint32_t tr = thr_row(P, u);
  if (tr != INF32) {
    uint32_t *trow = P.thr + (size_t)tr * P.cap + cu;
    for (uint32_t i = lane; i < m; i += WAVE) trow[i] = rank_of(s_tmp[i], L.rm);
  }
  const size_t base = (size_t)u * P.cap + cu;
  uint32_t x0, x1;  // the two smallest ranks of the level, for its record
  if (m <= (uint32_t)WAVE) {
    uint32_t x = (uint32_t)lane < m ? rank_of(s_tmp[lane], L.rm) : INF32;
    x = m <= COUNT_SORT_MAX ? wave_sort_few(x, m, s_cnt + (1 + KR) * WAVE) : wave_sort_reg(x);
    if ((uint32_t)lane < m) {
      P.sk_rank[base + lane] = x;
      P.sk_dist[base + lane] = D;
    }
    x0 = __shfl(x, 0, WAVE);
    x1 = __shfl(x, 1, WAVE);
  } else {
    for (uint32_t i = lane; i < m; i += WAVE) s_id[i] = rank_of(s_tmp[i], L.rm);
    wave_sort_lds(s_id, m);  // m <= SB
    for (uint32_t i = lane; i < m; i += WAVE) {
      P.sk_rank[base + i] = s_id[i];
      P.sk_dist[base + i] = D;
    }
    x0 = s_id[0];
    x1 = s_id[1];
  }
#pragma unroll
  for (int g = 0; g < KR; ++g)
    if ((uint32_t)(64 * g + lane) < nset) P.bk[(size_t)u * P.k + 64 * g + lane] = set.v[g];
  if (lane == 0) {
    P.cnt[u] = cu + m;
    P.lvl[(size_t)(D % P.NS) * P.n + u] = level_record(D, x0, x1, cu, m);
    ctr_add(P, CF_COMMITS, 1);
  }
  if (mark) mark_neighbours<UNITW>(P, u, D);
  return true;
}

// One task, by one wave.  slot == INF32: the task is the whole vertex and
// commits; otherwise it leaves its kept set in scratch slot `slot`.
template <bool UNITW, int KR, uint32_t SB>
__device__ inline void ads_task(const AdsArgs &P, uint32_t D, uint32_t u, uint32_t sub, uint32_t slot,
                                uint32_t task_arcs, int sparse, int mark, uint32_t *s_id, uint32_t *s_tmp,
                                uint32_t *s_cnt) {
  const int lane = lane_id();
  if (sparse && sub == 0 && lane == 0) {
    const uint32_t sD = D % P.NS;
    atomicAnd(&P.flags[(size_t)u * P.FW + (sD >> 5)], ~(1u << (sD & 31)));
  }
  Level<KR> L;
  level_init(P, u, L, s_cnt);
  const uint64_t r0 = P.row_ptr[u], r1 = P.row_ptr[u + 1];
  uint64_t a0 = r0, a1 = r1;
  if (slot != INF32) {
    a0 = r0 + (uint64_t)sub * task_arcs;
    a1 = a0 + task_arcs < r1 ? a0 + task_arcs : r1;
  }
  const uint64_t examined = (sparse && P.plane && D >= P.flag_from)
                                ? gather_flagged<UNITW, KR, SB>(P, D, a0, a1, L, s_id, s_tmp, s_cnt)
                                                 : gather_arcs<UNITW, KR, SB>(P, D, a0, a1, L, s_id, s_tmp, s_cnt);
  if (lane == 0) {
    ctr_add(P, CF_EXAMINED, examined);
    ctr_add(P, CF_SURVIVORS, L.nsurv);
    ctr_add(P, CF_PRUNES, L.nprune);
  }
  if (P.dbg) {
    const uint64_t nm = wave_sum_u64(L.nmatch);
    if (lane == 0) {
      ctr_add(P, CF_SCANNED, a1 - a0);
      ctr_add(P, CF_MATCHED, nm);
    }
  }
  if (L.overflow) {
    if (lane == 0) atomicOr(&P.status[1], 1u);
    return;
  }
  if (slot == INF32) {
    level_commit<UNITW, KR>(P, u, D, L, mark, s_id, s_tmp, s_cnt);
  } else {
    uint32_t m = 0;
    if (L.ns) {
      KSet<KR> set = L.set0;
      uint32_t nset = L.nset0;
      m = prune_level(s_id, s_tmp, s_cnt, L.ns, P.k, L.rm, set, nset);
      for (uint32_t i = lane; i < m; i += WAVE) P.kept[(size_t)slot * SB + i] = s_tmp[i];
    }
    if (lane == 0) P.kept_cnt[slot] = m;
  }
}

// ---------------------------------------------------------------------------
// Two small tasks per wave (k <= 32, rounds run from worklists).  Lanes
// 0..31 run one task and lanes 32..63 the next; every step works within the
// lane's half (shuffles of width 32, ballots cut to the half), so the fixed
// per-task instructions are shared by two tasks.  A task the halves cannot
// finish -- a slice of a split vertex, a row of more than PAIR_ROW_MAX arcs,
// more than 64 survivors in its level -- is left to the one-wave kernel, which runs after this one in the same round
// (pend[t] = 1); it is left before it has written anything but its own flag
// bit, which that kernel clears again.  Tasks of a round are independent and
// the prune does not depend on how candidates are grouped, so both kernels
// give the same levels.
// ---------------------------------------------------------------------------
constexpr uint32_t HALF = 32;
// Rows longer than this go to the one-wave kernel too: a wave runs two
// unrelated tasks, and a long row would keep its partner half idle (2,048
// and 1,024 measured equal on the large weighted workload, 4,096 and no limit
// 2-4% slower).
constexpr uint64_t PAIR_ROW_MAX = 2048;
__device__ inline uint32_t half_lane() { return (uint32_t)lane_id() & (HALF - 1); }
__device__ inline uint32_t half_ballot(bool p) { return (uint32_t)(__ballot(p) >> ((uint32_t)lane_id() & HALF)); }
__device__ inline uint32_t half_below(uint32_t m) { return (uint32_t)__popc(m & ((1u << half_lane()) - 1u)); }
__device__ inline uint32_t half_shfl(uint32_t x, uint32_t src) { return __shfl(x, (int)src, HALF); }
__device__ inline uint32_t half_scan_incl(uint32_t x) {
  const uint32_t l = half_lane();
#pragma unroll
  for (int d = 1; d < (int)HALF; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, HALF);
    if (l >= (uint32_t)d) x += y;
  }
  return x;
}
// ascending sort of one value per lane within each half (bitonic network)
__device__ inline uint32_t half_sort(uint32_t x) {
  const uint32_t l = half_lane();
#pragma unroll
  for (uint32_t k2 = 2; k2 <= HALF; k2 <<= 1) {
#pragma unroll
    for (uint32_t j = k2 >> 1; j > 0; j >>= 1) {
      const uint32_t y = __shfl_xor(x, (int)j, HALF);
      const bool keep_min = ((l & k2) == 0) == ((l & j) == 0);
      x = keep_min ? (x < y ? x : y) : (x > y ? x : y);
    }
  }
  return x;
}
// a bitonic sequence within each half, ascending
__device__ inline uint32_t half_bitonic_merge(uint32_t x) {
  const uint32_t l = half_lane();
#pragma unroll
  for (uint32_t j = HALF / 2; j >= 1; j >>= 1) {
    const uint32_t y = __shfl_xor(x, (int)j, HALF);
    x = (l & j) == 0 ? (x < y ? x : y) : (x > y ? x : y);
  }
  return x;
}
// values below r (per lane) in the half's ascending set (INF32 above its size)
__device__ inline uint32_t half_count_below(uint32_t setv, uint32_t r) {
  uint32_t q = 0;
#pragma unroll
  for (uint32_t s = HALF / 2; s >= 1; s >>= 1) {
    const uint32_t val = half_shfl(setv, q + s - 1);
    if (val < r) q += s;
  }
  if (half_shfl(setv, q) < r) ++q;  // all 32 below r
  return q;
}

// 6 waves per SIMD (80 registers, a few spilled) measured 2% faster than 5 on
// the large weighted workload; 8 (64 registers) slower
template <bool UNITW>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(6, 8)))
void k_ads_pairs(AdsArgs P, uint32_t D, const uint32_t *task_u, const uint32_t *task_sub, const uint32_t *task_slot,
                 const uint64_t *d_ntasks, uint8_t *pend) {
  __shared__ uint32_t s_id[2][2 * HALF];            // survivors of the level (ids)
  __shared__ uint32_t s_acc[2][2 * HALF];           // accepted ids, in id order
  __shared__ uint32_t s_set[2][HALF];               // the set at the level start
  __shared__ __align__(16) uint32_t s_r[2][HALF];   // chunk ranks
  const uint32_t lane = (uint32_t)lane_id(), h = lane >> 5, hl = lane & (HALF - 1);
  const uint32_t k = P.k;
  const uint64_t total = *d_ntasks;
  const bool flagged = P.plane && D >= P.flag_from;
  for (uint64_t pi = blockIdx.x; 2 * pi < total; pi += gridDim.x) {
    const uint64_t t = 2 * pi + h;
    const bool live = t < total;
    uint32_t u = 0, slot = INF32;
    if (live) {
      u = task_u[t];
      slot = task_slot[t];
    }
    bool defer = live && slot != INF32;  // a slice of a split vertex
    bool act = live && !defer;           // half-uniform from here on
    if (act && hl == 0) {
      const uint32_t sD = D % P.NS;
      atomicAnd(&P.flags[(size_t)u * P.FW + (sD >> 5)], ~(1u << (sD & 31)));
    }
    const RankMap rm = rank_map(P.seg[seg_of(P.gid, u)]);
    const uint32_t cu = act ? P.cnt[u] : 0u;
    const uint32_t nset0 = cu < k ? cu : k;
    const uint32_t setv = (act && hl < nset0) ? P.bk[(size_t)u * k + hl] : INF32;
    s_set[h][hl] = setv;
    wave_lds_sync();
    const bool full0 = nset0 == k;
    const uint32_t set_kth = half_shfl(setv, k - 1);
    const uint32_t T0 = full0 ? set_kth : INF32;
    uint32_t ns = 0;
    uint64_t examined = 0;
    // one candidate per lane: kept if below T0 and not in the start set
    auto offer = [&](bool valid, uint32_t r) {
      bool pass = act && valid && (!full0 || r < T0);
      if (pass) {
        uint32_t lo = 0, hi = nset0;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_set[h][mid] < r) lo = mid + 1;
          else hi = mid;
        }
        if (lo < nset0 && s_set[h][lo] == r) pass = false;
      }
      const uint32_t m = half_ballot(pass);
      const uint32_t np = (uint32_t)__popc(m);
      if (ns + np > 2 * HALF) {
        defer = true;  // more survivors than one chunk: the one-wave kernel
        act = false;
      } else {
        if (pass) s_id[h][ns + half_below(m)] = id_of(r, rm);
        ns += np;
      }
      wave_lds_sync();
    };
    // one in-arc per lane: the level its tail committed at D - w
    auto batch = [&](bool valid, uint64_t a) {
      uint32_t v = 0, st = 0, cn = 0, r0 = INF32, r1 = INF32;
      if (act && valid) {
        v = P.col[a];
        const uint32_t wv = UNITW ? 1u : P.w[a];
        if (wv <= D) {
          const uint32_t src = D - wv;
          const uint4 rec = P.lvl[(size_t)(src % P.NS) * P.n + v];
          if (rec.x == src && (!full0 || rec.y < T0)) {
            r0 = rec.y;
            r1 = rec.z;
            st = rec.w & 0xFFFFu;
            cn = rec.w >> 16;
          }
        }
      }
      const bool one = cn != 0 && cn <= 2, two = cn == 2;
      examined += (uint32_t)__popc(half_ballot(one)) + (uint32_t)__popc(half_ballot(two));
      offer(one, r0);
      offer(two, r1);
      // long lists: one at a time per half, 32 entries per step; a level is
      // stored in increasing rank order, so once a rank reaches T0 the rest
      // of the list cannot enter
      uint32_t lm = half_ballot(act && cn >= LONG_LIST);
      while (__ballot(lm != 0)) {
        const bool has = lm != 0;
        const uint32_t j = has ? (uint32_t)(__ffs(lm) - 1) : 0u;
        if (has) lm &= lm - 1;
        const uint32_t vj = half_shfl(v, j), stj = half_shfl(st, j);
        uint32_t cnj = half_shfl(cn, j);
        if (!has) cnj = 0;
        const uint32_t *lst = P.sk_rank + (size_t)vj * P.cap + stj;
        bool go = has;
        for (uint32_t c0 = 0;; c0 += HALF) {
          const bool step = go && act && c0 < cnj;
          if (!__ballot(step)) break;
          const uint32_t i = c0 + hl;
          const bool ok = step && i < cnj;
          const uint32_t r = ok ? lst[i] : INF32;
          if (step) examined += cnj - c0 < HALF ? cnj - c0 : HALF;
          offer(ok, r);
          if (full0 && half_ballot(ok && r >= T0)) go = false;
        }
      }
      const uint32_t cs = (act && cn > 2 && cn < LONG_LIST) ? cn : 0u;
      const uint32_t incl = half_scan_incl(cs);
      const uint32_t tot = half_shfl(incl, HALF - 1);
      const uint32_t excl = incl - cs;
      examined += tot;
      for (uint32_t c0 = 0;; c0 += HALF) {
        const bool cm = act && c0 < tot;
        if (!__ballot(cm)) break;
        const uint32_t idx = c0 + hl;
        uint32_t pos = 0;  // owner lane: first lane whose inclusive count exceeds idx
#pragma unroll
        for (uint32_t s = HALF / 2; s >= 1; s >>= 1) {
          const uint32_t val = half_shfl(incl, pos + s - 1);
          if (val <= idx) pos += s;
        }
        const bool ok = cm && idx < tot;
        const uint32_t ov = half_shfl(v, pos), ost = half_shfl(st, pos), oex = half_shfl(excl, pos);
        uint32_t r = INF32;
        if (ok) r = P.sk_rank[(size_t)ov * P.cap + ost + (idx - oex)];
        offer(ok, r);
      }
    };
    uint64_t a0 = 0, a1 = 0;
    if (act) {
      a0 = P.row_ptr[u];
      a1 = P.row_ptr[u + 1];
      if (a1 - a0 > PAIR_ROW_MAX) {
        defer = true;  // a long row: the one-wave kernel
        act = false;
      }
    }
    if (flagged) {
      // only the arcs flagged in this round's plane
      const uint32_t *plane = P.plane + (size_t)(D % P.NS) * P.pw;
      const uint64_t w0 = a0 >> 5, w1 = (a1 + 31) >> 5;
      for (uint64_t wb = w0;; wb += HALF) {
        const bool more = act && wb < w1;
        if (!__ballot(more)) break;
        const uint64_t wi = wb + hl;
        uint32_t bits = 0;
        if (more && wi < w1) {
          bits = plane[wi];
          const uint64_t base = wi << 5;
          if (base < a0) bits &= ~0u << (uint32_t)(a0 - base);
          if (a1 - base < 32) bits &= (1u << (uint32_t)(a1 - base)) - 1u;
        }
        const uint32_t incl = half_scan_incl((uint32_t)__popc(bits));
        const uint32_t tot = half_shfl(incl, HALF - 1);
        for (uint32_t c0 = 0;; c0 += HALF) {
          const bool cm = act && more && c0 < tot;
          if (!__ballot(cm)) break;
          const uint32_t idx = c0 + hl;
          uint32_t pos = 0;  // word (lane) holding set bit idx
#pragma unroll
          for (uint32_t s = HALF / 2; s >= 1; s >>= 1) {
            const uint32_t val = half_shfl(incl, pos + s - 1);
            if (val <= idx) pos += s;
          }
          const bool ok = cm && idx < tot;
          const uint32_t src = ok ? pos : 0u;
          uint32_t x = half_shfl(bits, src);
          uint32_t kth = idx - (half_shfl(incl, src) - (uint32_t)__popc(x));
          uint32_t bit = 0;
#pragma unroll
          for (uint32_t sh = 16; sh >= 1; sh >>= 1) {
            const uint32_t cnt = (uint32_t)__popc(x & ((1u << sh) - 1u));
            if (kth >= cnt) {
              kth -= cnt;
              x >>= sh;
              bit += sh;
            }
          }
          batch(ok, ((wb + src) << 5) + bit);
        }
      }
    } else {
      for (uint64_t b = a0;; b += HALF) {
        const bool more = act && b < a1;
        if (!__ballot(more)) break;
        batch(more && b + hl < a1, b + hl);
      }
    }
    // Up to 64 survivors, sorted by id and decided in chunks of 32: each id
    // is accepted if fewer than k ranks below its own are in the set (which
    // by the second chunk holds the first chunk's accepted ranks) or among
    // the chunk's earlier candidates.  (Every shuffle here runs on all lanes:
    // a lane reads another only while that lane is active.)
    const bool two = __ballot(act && ns > HALF) != 0;  // some half has a second chunk
    uint32_t lo = half_sort((act && hl < ns) ? s_id[h][hl] : INF32), hi = INF32;
    if (two) {
      const uint32_t xb = half_sort((act && HALF + hl < ns) ? s_id[h][HALF + hl] : INF32);
      const uint32_t xbr = half_shfl(xb, HALF - 1 - hl);
      const uint32_t l2 = lo < xbr ? lo : xbr, h2 = lo < xbr ? xbr : lo;
      lo = half_bitonic_merge(l2);  // the 32 smallest ids
      hi = half_bitonic_merge(h2);  // the next 32
    }
    // one chunk against the set (setc, nsetc); prevx: the id before the chunk
    auto decide = [&](uint32_t x, uint32_t prevx, uint32_t setc, uint32_t nsetc, uint32_t &r_out) -> bool {
      uint32_t left = __shfl_up(x, 1, HALF);
      if (hl == 0) left = prevx;
      bool valid = act && x != INF32 && x != left;
      const uint32_t r = valid ? rank_of(x, rm) : INF32;
      const uint32_t q = half_count_below(setc, r);
      const uint32_t atq = half_shfl(setc, q < HALF - 1 ? q : HALF - 1);
      if (q < nsetc && atq == r) valid = false;
      const uint32_t vm = half_ballot(valid);
      s_r[h][hl] = valid ? r : INF32;
      wave_lds_sync();
      uint32_t top = vm ? 32u - (uint32_t)__clz(vm) : 0u;
      const uint32_t top2 = __shfl_xor(top, (int)HALF, WAVE);
      top = top > top2 ? top : top2;
      uint32_t cp = 0;
      for (uint32_t j4 = 0; j4 < top; j4 += 4) {
        const uint4 vv = *reinterpret_cast<const uint4 *>(&s_r[h][j4]);
        cp += (j4 + 0 < hl && vv.x < r) ? 1u : 0u;
        cp += (j4 + 1 < hl && vv.y < r) ? 1u : 0u;
        cp += (j4 + 2 < hl && vv.z < r) ? 1u : 0u;
        cp += (j4 + 3 < hl && vv.w < r) ? 1u : 0u;
      }
      wave_lds_sync();  // s_r is rewritten by the next chunk
      r_out = r;
      return valid && q + cp < k;
    };
    // the set after a chunk: the k smallest of the set and the chunk's
    // accepted ranks (xs, ascending)
    auto merge_set = [&](uint32_t setc, uint32_t xs) -> uint32_t {
      const uint32_t xrev = half_shfl(xs, HALF - 1 - hl);
      const uint32_t mm = half_bitonic_merge(setc < xrev ? setc : xrev);
      return hl < k ? mm : INF32;
    };
    uint32_t r1 = INF32;
    const bool acc1 = decide(lo, INF32, setv, nset0, r1);
    const uint32_t am1 = half_ballot(acc1);
    const uint32_t m1 = (uint32_t)__popc(am1);
    if (acc1) s_acc[h][half_below(am1)] = lo;
    const uint32_t xs1 = half_sort(acc1 ? r1 : INF32);
    uint32_t set1 = merge_set(setv, xs1);
    uint32_t nset1 = nset0 + m1 < k ? nset0 + m1 : k;
    uint32_t ra = xs1, rb = INF32, m = m1;  // the level's ranks ascending: ra, then rb
    if (two) {
      const uint32_t prevx = half_shfl(lo, HALF - 1);  // the first chunk is full when there is a second
      uint32_t r2 = INF32;
      const bool acc2 = decide(hi, prevx, set1, nset1, r2);
      const uint32_t am2 = half_ballot(acc2);
      const uint32_t m2 = (uint32_t)__popc(am2);
      if (acc2) s_acc[h][m1 + half_below(am2)] = hi;
      const uint32_t xs2 = half_sort(acc2 ? r2 : INF32);
      set1 = merge_set(set1, xs2);
      nset1 = nset1 + m2 < k ? nset1 + m2 : k;
      const uint32_t x2r = half_shfl(xs2, HALF - 1 - hl);
      const uint32_t l2 = xs1 < x2r ? xs1 : x2r, h2 = xs1 < x2r ? x2r : xs1;
      ra = half_bitonic_merge(l2);
      rb = half_bitonic_merge(h2);
      m = m1 + m2;
    }
    wave_lds_sync();  // s_acc is read below
    const uint32_t x0 = half_shfl(ra, 0), x1 = half_shfl(ra, 1);
    bool committed = false;
    if (act && m) {
      if (cu + m > P.cap) {
        if (hl == 0) atomicOr(&P.status[0], 1u);
      } else {
        committed = true;
        const uint32_t tr = thr_row(P, u);
        if (tr != INF32) {
          uint32_t *trow = P.thr + (size_t)tr * P.cap + cu;
          if (hl < m) trow[hl] = rank_of(s_acc[h][hl], rm);
          if (HALF + hl < m) trow[HALF + hl] = rank_of(s_acc[h][HALF + hl], rm);
        }
        const size_t base = (size_t)u * P.cap + cu;
        if (hl < m) {
          P.sk_rank[base + hl] = ra;
          P.sk_dist[base + hl] = D;
        }
        if (HALF + hl < m) {
          P.sk_rank[base + HALF + hl] = rb;
          P.sk_dist[base + HALF + hl] = D;
        }
        if (hl < nset1) P.bk[(size_t)u * k + hl] = set1;
        if (hl == 0) {
          P.cnt[u] = cu + m;
          P.lvl[(size_t)(D % P.NS) * P.n + u] = level_record(D, x0, x1, cu, m);
        }
      }
    }
    // the heads of u's out-arcs are queued for round D + w
    uint64_t b0 = 0, b1 = 0;
    if (committed) {
      b0 = P.out_ptr[u];
      b1 = P.out_ptr[u + 1];
    }
    for (uint64_t b = b0;; b += HALF) {
      const bool more = committed && b < b1;
      if (!__ballot(more)) break;
      const uint64_t a = b + hl;
      const bool want = more && a < b1;
      uint32_t y = 0, s = 0;
      if (want) {
        y = P.out_col[a];
        const uint32_t wv = UNITW ? 1u : P.out_w[a];
        s = (D + wv) % P.NS;
        if (P.plane && D >= P.plane_from) {
          const uint32_t p = P.out_to_in[a];
          atomicOr(&P.plane[(size_t)s * P.pw + (p >> 5)], 1u << (p & 31));
        }
      }
      mark_targets<UNITW>(P, want, y, s);
    }
    if (live && hl == 0) {
      pend[t] = defer ? 1 : 0;
      if (!defer) {
        ctr_add(P, CF_EXAMINED, examined);
        ctr_add(P, CF_SURVIVORS, ns);
        if (committed) ctr_add(P, CF_COMMITS, 1);
      }
    }
    wave_lds_sync();  // the half buffers are rewritten by the next pair
  }
}

// One wave per task.  task_slot == INF32: the task is the whole vertex and
// commits; otherwise it leaves its kept set in scratch slot task_slot.  With
// d_ntasks (device) the grid strides over that many tasks (the host does not
// know the count); otherwise one wave per task.  With `only`, just the tasks
// t with only[t] != 0 (those the two-task kernel left).
template <bool UNITW, int KR, uint32_t SB>
__global__ __launch_bounds__(TASK_WPB * WAVE) __attribute__((amdgpu_waves_per_eu(SB <= ADS_SB / 2 ? 5 : 4)))
void k_ads_tasks(AdsArgs P, uint32_t D, const uint32_t *task_u, const uint32_t *task_sub, const uint32_t *task_slot,
                 uint32_t ntasks, const uint64_t *d_ntasks, uint32_t task_arcs, int sparse, int mark,
                 const uint8_t *only) {
  __shared__ uint32_t lds_id[TASK_WPB][SB];
  __shared__ uint32_t lds_tmp[TASK_WPB][SB];
  __shared__ __align__(16) uint32_t lds_cnt[TASK_WPB][(2 + KR) * WAVE];
  const int wv = threadIdx.x / WAVE;
  const uint64_t total = d_ntasks ? *d_ntasks : ntasks;
  for (uint64_t item = (uint64_t)blockIdx.x * TASK_WPB + wv; item < total; item += (uint64_t)gridDim.x * TASK_WPB) {
    if (only && !only[item]) continue;  // done by the two-task kernel
    ads_task<UNITW, KR, SB>(P, D, task_u[item], task_sub[item], task_slot[item], task_arcs, sparse, mark, lds_id[wv],
                            lds_tmp[wv], lds_cnt[wv]);
  }
}

// One block per split vertex: MERGE_WPB - 1 waves each prune the union of a
// strided share of its tasks' kept sets into a partial set in LDS, then the
// first wave prunes the union of the partial sets and commits.  The prune is
// associative and idempotent, so the grouping does not change the result;
// it shortens the chain of dependent work per hub, which bounds a round.
constexpr int MERGE_WPB = 8;
template <bool UNITW, int KR, uint32_t SB>
__global__ __launch_bounds__(MERGE_WPB * WAVE) void k_ads_merge(AdsArgs P, uint32_t D, const uint32_t *split_u,
                                                                const uint32_t *split_first,
                                                                const uint32_t *split_nt, uint32_t nsplit,
                                                                const uint64_t *d_nsplit, int mark) {
  constexpr uint32_t NW = MERGE_WPB - 1;  // waves that build partial sets
  __shared__ uint32_t lds_id[MERGE_WPB][SB];
  __shared__ uint32_t lds_tmp[MERGE_WPB][SB];
  __shared__ __align__(16) uint32_t lds_cnt[MERGE_WPB][(2 + KR) * WAVE];
  __shared__ uint32_t part_n[MERGE_WPB];
  __shared__ uint32_t s_mark;  // the item committed a level: its out-arcs are marked
  const int lane = lane_id();
  const int wv = threadIdx.x / WAVE;
  uint32_t *s_id = lds_id[wv];
  uint32_t *s_tmp = lds_tmp[wv];
  uint32_t *s_cnt = lds_cnt[wv];
  // the block's split vertices (uniform over the block): every wave reaches
  // both barriers of every item
  const uint64_t total = d_nsplit ? *d_nsplit : nsplit;
  for (uint64_t item = blockIdx.x; item < total; item += gridDim.x) {
    const uint32_t u = split_u[item];
    const uint32_t first = split_first[item];
    const uint32_t nt = split_nt[item];
    Level<KR> L;
    level_init(P, u, L, s_cnt);
    if (wv > 0) {
      // tasks wv - 1, wv - 1 + NW, ...: a virtual list of `mine` tasks
      const uint32_t t0 = (uint32_t)wv - 1;
      const uint32_t mine = nt > t0 ? (nt - t0 + NW - 1) / NW : 0u;
      for (uint32_t g0 = 0; g0 < mine && !L.overflow; g0 += WAVE) {
        const uint32_t task = first + t0 + (g0 + lane) * NW;
        const uint32_t cn = g0 + lane < mine ? P.kept_cnt[task] : 0u;
        const uint32_t incl = wave_scan_incl(cn);
        const uint32_t tot = __shfl(incl, WAVE - 1, WAVE);
        const uint32_t excl = incl - cn;
        for (uint32_t c0 = 0; c0 < tot && !L.overflow; c0 += WAVE) {
          const uint32_t idx = c0 + lane;
          uint32_t pos = 0;
#pragma unroll
          for (uint32_t sh = 32; sh >= 1; sh >>= 1) {
            const uint32_t val = __shfl(incl, (int)(pos + sh - 1), WAVE);
            if (val <= idx) pos += sh;
          }
          const bool valid = idx < tot;
          const uint32_t oex = __shfl(excl, (int)pos, WAVE);
          const uint32_t otask = __shfl(task, (int)pos, WAVE);
          uint32_t id = INF32, r = INF32;
          if (valid) {
            id = P.kept[(size_t)otask * SB + (idx - oex)];
            r = rank_of(id, L.rm);
          }
          level_offer<KR, SB>(P, L, valid, r, true, id, s_id, s_tmp, s_cnt);
        }
      }
      uint32_t m = 0;
      if (!L.overflow && L.ns) {
        KSet<KR> set = L.set0;
        uint32_t nset = L.nset0;
        m = prune_level(s_id, s_tmp, s_cnt, L.ns, P.k, L.rm, set, nset);  // partial set in s_tmp[0..m)
      }
      if (lane == 0) part_n[wv] = L.overflow ? INF32 : m;
    }
    __syncthreads();
    if (wv == 0) {
      for (int w = 1; w < MERGE_WPB && !L.overflow; ++w) {
        const uint32_t pn = part_n[w];
        if (pn == INF32) {
          L.overflow = true;
          break;
        }
        const uint32_t *part = lds_tmp[w];
        for (uint32_t c0 = 0; c0 < pn && !L.overflow; c0 += WAVE) {
          const bool valid = c0 + lane < pn;
          const uint32_t id = valid ? part[c0 + lane] : INF32;
          const uint32_t r = valid ? rank_of(id, L.rm) : INF32;
          level_offer<KR, SB>(P, L, valid, r, true, id, s_id, s_tmp, s_cnt);
        }
      }
      bool committed = false;
      if (L.overflow) {
        if (lane == 0) atomicOr(&P.status[1], 1u);
      } else {
        committed = level_commit<UNITW, KR>(P, u, D, L, 0, s_id, s_tmp, s_cnt);
      }
      if (lane == 0) s_mark = committed && mark ? 1u : 0u;
    }
    // the partial sets are read before the next item rebuilds them; s_mark is
    // read by every wave before wave 0 passes the next item's first barrier
    __syncthreads();
    // a split vertex is a hub: every wave of the block marks a share of its out-arcs
    if (s_mark) mark_neighbours<UNITW>(P, u, D, (uint32_t)wv, MERGE_WPB);
  }
}

// Last pass over the rows with a threshold row (one wave per row): the row
// holds the sketch in canonical (distance, id) order (written at commit); it
// is copied into the sketch row, and entry j of the threshold row becomes
// T_j = the k-th smallest rank of entries 0..j-1 (0 for j < k, meaning 2^32).
// Every later entry ranks below its T_j (that is what membership of the
// sketch means), so each one enters the running bottom-k set and evicts its
// maximum, and no later entry is above that maximum.  Hence for a chunk C of
// up to 64 entries after a full set S, the threshold of the chunk's i-th
// entry is the (i+1)-th largest of S and C together, and the next S is the k
// smallest of them: one sort and a few bitonic merges per chunk.  The set is
// held in KR registers per lane (k <= 64 KR).
template <int KR>
__global__ __launch_bounds__(256) void k_hip_thresholds(uint32_t rows, const uint32_t *row_vertex, uint32_t cap,
                                                        uint32_t k, const uint32_t *cnt, uint32_t *sk_rank,
                                                        uint32_t *thr) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (row >= rows) return;
  const uint32_t u = row_vertex ? row_vertex[row] : (uint32_t)row;
  const uint32_t c = cnt[u];
  uint32_t *rk = sk_rank + (size_t)u * cap;
  uint32_t *out = thr + (size_t)row * cap;  // canonical ranks in, thresholds out (each lane its own slots)
  const uint32_t k0 = c < k ? c : k;
  uint32_t first[KR];
#pragma unroll
  for (int g = 0; g < KR; ++g) {
    const uint32_t e = 64u * g + lane;
    first[g] = e < k0 ? out[e] : INF32;
    if (e < k0) {
      rk[e] = first[g];
      out[e] = 0;
    }
  }
  if (c <= k) return;
  // S: the first k entries, ascending, INF32 above k
  KSet<KR> S;
  if (KR == 1) {
    S.v[0] = wave_sort_reg(first[0]);
  } else {
    uint32_t hi;
    wave_merge2(wave_sort_reg(first[0]), wave_sort_reg(first[KR - 1]), S.v[0], hi);
    S.v[KR - 1] = hi;
  }
  for (uint32_t j0 = k; j0 < c; j0 += WAVE) {
    const uint32_t m = c - j0 < (uint32_t)WAVE ? c - j0 : (uint32_t)WAVE;
    const uint32_t mine = lane < m ? out[j0 + lane] : INF32;
    if (lane < m) rk[j0 + lane] = mine;
    const uint32_t ca = wave_sort_reg(mine);  // chunk ascending, INF32 above m
    // the 64 largest: S descending (0 past its size) against C ascending (0 below 64 - m)
    const uint32_t sd = kset_at(S, lane < k ? k - 1 - lane : 0u);
    const uint32_t cs = __shfl(ca, (int)(lane >= WAVE - m ? lane - (WAVE - m) : 0), WAVE);
    uint32_t top = (lane < k ? sd : 0u) > (lane >= WAVE - m ? cs : 0u) ? (lane < k ? sd : 0u)
                                                                        : (lane >= WAVE - m ? cs : 0u);
    top = wave_bitonic_merge(top, true);  // lane i: the (i+1)-th largest
    if (lane < m) out[j0 + lane] = top;
    kset_merge(S, ca, k);  // the k smallest of S and C
  }
}

// ---------------------------------------------------------------------------
// task lists
// ---------------------------------------------------------------------------
// count: entries the grid covers; d_count (device, may be null): the list's
// length when only the device knows it (entries past it count zero tasks)
__global__ void k_task_count(const uint32_t *list, uint32_t count, const uint32_t *d_count, const uint64_t *row_ptr,
                             uint32_t task_arcs, uint32_t *ntask, uint32_t *nslot, uint32_t *isplit) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (d_count && i >= *d_count) {
    ntask[i] = nslot[i] = isplit[i] = 0;
    return;
  }
  const uint32_t u = list[i];
  const uint64_t d = row_ptr[u + 1] - row_ptr[u];
  const uint32_t nt = d <= task_arcs ? 1u : (uint32_t)((d + task_arcs - 1) / task_arcs);
  ntask[i] = nt;
  nslot[i] = nt > 1 ? nt : 0u;
  isplit[i] = nt > 1 ? 1u : 0u;
}

__global__ void k_task_fill(const uint32_t *list, uint32_t count, const uint32_t *d_count, const uint32_t *ntask,
                            const uint64_t *task_off, const uint64_t *slot_off, const uint64_t *split_off,
                            uint32_t *task_u, uint32_t *task_sub, uint32_t *task_slot, uint32_t *split_u,
                            uint32_t *split_first, uint32_t *split_nt) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || (d_count && i >= *d_count)) return;
  const uint32_t u = list[i];
  const uint32_t nt = ntask[i];
  const uint64_t t0 = task_off[i];
  for (uint32_t j = 0; j < nt; ++j) {
    task_u[t0 + j] = u;
    task_sub[t0 + j] = j;
    task_slot[t0 + j] = nt > 1 ? (uint32_t)(slot_off[i] + j) : INF32;
  }
  if (nt > 1) {
    const uint64_t s = split_off[i];
    split_u[s] = u;
    split_first[s] = (uint32_t)slot_off[i];
    split_nt[s] = nt;
  }
}

struct TaskList {
  uint32_t *task_u, *task_sub, *task_slot;
  uint32_t *split_u, *split_first, *split_nt;
  uint32_t ntasks = 0, nsplit = 0, nslots = 0;
  uint32_t task_arcs = TASK_ARCS;  // arcs per task of a split vertex
};

// scratch of build_tasks: 3 count arrays + 3 offset arrays
struct TaskScratch {
  uint32_t *ntask, *nslot, *isplit;
  uint64_t *toff, *soff, *poff;
};

// The task list of a worklist whose length only the device knows: each
// 256-thread block takes TB_ITEMS consecutive entries per thread and reserves
// the tile's tasks, kept slots and split records with one atomic per counter
// (the order of the tasks does not matter: the prune does not depend on it).
// tot: [0] tasks, [1] kept slots, [2] split vertices, zero before the launch.
constexpr uint32_t TB_ITEMS = 4;
__global__ __launch_bounds__(256) void k_task_build(const uint32_t *list, const uint32_t *d_count,
                                                    const uint64_t *row_ptr, uint32_t task_arcs, uint64_t *tot,
                                                    uint32_t *task_u, uint32_t *task_sub, uint32_t *task_slot,
                                                    uint32_t *split_u, uint32_t *split_first, uint32_t *split_nt) {
  __shared__ uint32_t wsum[3][4];
  __shared__ uint64_t base[3];
  const uint32_t lane = (uint32_t)lane_id(), wv = threadIdx.x / WAVE;
  const uint32_t count = *d_count;
  constexpr uint32_t TILE = 256 * TB_ITEMS;
  for (uint64_t b = (uint64_t)blockIdx.x * TILE; b < count; b += (uint64_t)gridDim.x * TILE) {
    uint32_t u[TB_ITEMS], nt[TB_ITEMS];
    uint32_t c[3] = {0, 0, 0};
#pragma unroll
    for (uint32_t j = 0; j < TB_ITEMS; ++j) {
      const uint64_t i = b + (uint64_t)threadIdx.x * TB_ITEMS + j;
      u[j] = 0;
      nt[j] = 0;
      if (i < count) {
        u[j] = list[i];
        const uint64_t d = row_ptr[u[j] + 1] - row_ptr[u[j]];
        nt[j] = d <= task_arcs ? 1u : (uint32_t)((d + task_arcs - 1) / task_arcs);
      }
      c[0] += nt[j];
      c[1] += nt[j] > 1 ? nt[j] : 0u;
      c[2] += nt[j] > 1 ? 1u : 0u;
    }
    uint32_t incl[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      incl[q] = wave_scan_incl(c[q]);
      if (lane == WAVE - 1) wsum[q][wv] = incl[q];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      const uint32_t q = threadIdx.x;
      const uint32_t t = wsum[q][0] + wsum[q][1] + wsum[q][2] + wsum[q][3];
      base[q] = t ? atomicAdd((unsigned long long *)&tot[q], (unsigned long long)t) : 0ull;
    }
    __syncthreads();
    uint64_t off[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      uint64_t o = base[q] + (incl[q] - c[q]);
      for (uint32_t w = 0; w < wv; ++w) o += wsum[q][w];
      off[q] = o;
    }
    __syncthreads();  // wsum and base are rewritten by the next tile
#pragma unroll
    for (uint32_t j = 0; j < TB_ITEMS; ++j) {
      for (uint32_t t = 0; t < nt[j]; ++t) {
        task_u[off[0] + t] = u[j];
        task_sub[off[0] + t] = t;
        task_slot[off[0] + t] = nt[j] > 1 ? (uint32_t)(off[1] + t) : INF32;
      }
      if (nt[j] > 1) {
        split_u[off[2]] = u[j];
        split_first[off[2]] = (uint32_t)off[1];
        split_nt[off[2]] = nt[j];
        off[1] += nt[j];
        off[2] += 1;
      }
      off[0] += nt[j];
    }
  }
}

// task_arcs >= TASK_ARCS: the scratch slots are sized for TASK_ARCS
static void build_tasks(Ctx &c, const Graph &g, const uint32_t *list, uint32_t count, uint32_t task_arcs,
                        TaskScratch &ts, TaskList &tl) {
  tl.ntasks = tl.nsplit = tl.nslots = 0;
  tl.task_arcs = task_arcs;
  if (count == 0) return;
  const uint32_t blocks = (uint32_t)ceil_div(count, 256);
  k_task_count<<<blocks, 256, 0, c.s>>>(list, count, nullptr, g.in_ptr, task_arcs, ts.ntask, ts.nslot, ts.isplit);
  FL_LAUNCH_CHECK();
  scan_u32_to_u64(c, ts.ntask, ts.toff, count);
  scan_u32_to_u64(c, ts.nslot, ts.soff, count);
  scan_u32_to_u64(c, ts.isplit, ts.poff, count);
  k_task_fill<<<blocks, 256, 0, c.s>>>(list, count, nullptr, ts.ntask, ts.toff, ts.soff, ts.poff, tl.task_u,
                                        tl.task_sub, tl.task_slot, tl.split_u, tl.split_first, tl.split_nt);
  FL_LAUNCH_CHECK();
  uint64_t h[3];
  FL_HIP(hipMemcpyAsync(&h[0], ts.toff + count, 8, hipMemcpyDeviceToHost, c.s));
  FL_HIP(hipMemcpyAsync(&h[1], ts.soff + count, 8, hipMemcpyDeviceToHost, c.s));
  FL_HIP(hipMemcpyAsync(&h[2], ts.poff + count, 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  tl.ntasks = (uint32_t)h[0];
  tl.nslots = (uint32_t)h[1];
  tl.nsplit = (uint32_t)h[2];
}

// Undirected graph: the position of each arc (v, y) within row y, i.e. of the
// reverse arc (y, v) (rows are sorted and free of repeats, validated).
__global__ void k_reverse_arcs(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                               uint32_t *out_to_in) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m; a += stride) {
    uint32_t lo = 0, hi = n;  // tail: row_ptr[lo] <= a < row_ptr[hi]
    while (hi - lo > 1) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (row_ptr[mid] <= a) lo = mid;
      else hi = mid;
    }
    const uint32_t y = col[a];
    uint64_t b0 = row_ptr[y], b1 = row_ptr[y + 1];  // first position in row y with col >= lo
    while (b0 < b1) {
      const uint64_t mid = b0 + ((b1 - b0) >> 1);
      if (col[mid] < lo) b0 = mid + 1;
      else b1 = mid;
    }
    out_to_in[a] = (uint32_t)b0;
  }
}

// Work still pending after a round of a chunk (every worklist slot) and the
// round's task count, for the host's readback at the end of the chunk.
__global__ void k_round_pending(const uint32_t *wl_cnt, uint32_t NS, const uint64_t *d_ntasks, uint64_t *pend,
                                uint64_t *tasks) {
  uint64_t sum = 0;
  for (uint32_t s = threadIdx.x; s < NS; s += WAVE) sum += wl_cnt[s * CNT_PAD];
  sum = wave_sum_u64(sum);
  if (threadIdx.x == 0) {
    *pend = sum;
    *tasks = *d_ntasks;
  }
}

// list of vertices with at least one in-arc
__global__ void k_nonisolated_flags(uint32_t n, const uint64_t *row_ptr, uint32_t *flag) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = row_ptr[i + 1] > row_ptr[i] ? 1u : 0u;
}
__global__ void k_compact(uint32_t n, const uint32_t *flag, const uint64_t *pos, uint32_t *out) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (uint32_t)i;
}
// number of scratch slots a vertex needs when split
__global__ void k_slot_need(uint32_t n, const uint64_t *row_ptr, uint32_t *need) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const uint64_t d = row_ptr[i + 1] - row_ptr[i];
    need[i] = d > TASK_ARCS ? (uint32_t)((d + TASK_ARCS - 1) / TASK_ARCS) : 0u;
  }
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

size_t ads_scratch_bytes(uint32_t n, uint64_t m, uint32_t k, uint32_t NS) {
  const size_t FW = (NS + 31) / 32;
  const uint64_t slots = 2 * (m / TASK_ARCS) + 2;  // >= sum of ceil(deg/TASK_ARCS) over vertices with deg > TASK_ARCS
  const uint64_t tasks = (uint64_t)n + m / TASK_ARCS + 64;
  size_t b = 0;
  b += (size_t)n * k * 4;                  // bottom-k sets
  b += (size_t)NS * n * (16 + 4);          // per-slot level records + worklists
  b += (size_t)m * 4 + (size_t)NS * (m / 32 + 2) * 4;  // reverse-arc positions, arc bit planes
  b += (size_t)n * FW * 4;                 // worklist flags
  b += (size_t)NS * CNT_PAD * 4;           // worklist lengths, one per line
  b += (size_t)slots * (ADS_SB * (k > 64 ? 2 : 1) + 1) * 4;   // kept sets of split tasks
  b += (size_t)tasks * 4 * 3 * 2 + (size_t)n * 4 * 3 * 2;  // two task lists
  b += (size_t)n * (4 * 3 + 8 * 3) + (size_t)n * 24;       // task scratch, dense list
  b += (size_t)tasks;                      // tasks left by the two-task kernel
  b += (size_t)8 << 20;
  return b;
}

// Builds the sketches.  Returns FL_OK, or FL_ENOMEM / FL_ENOTIMPL.  The
// caller provides cap; on capacity overflow the call reports *need_more.
// Launches of the round kernels: the instance is picked by unit weights, the
// set registers of k and the survivor buffer of the build.
static void launch_tasks(hipStream_t s, uint32_t grid, bool unit, uint32_t k, uint32_t sb, const AdsArgs &P,
                         uint32_t D, const uint32_t *tu, const uint32_t *tsub, const uint32_t *tslot, uint32_t nt,
                         const uint64_t *dnt, uint32_t task_arcs, int sparse, int mark,
                         const uint8_t *only = nullptr) {
#define FL_TASKS(U, K, S)                                                                                          \
  k_ads_tasks<U, K, S><<<grid, TASK_WPB * WAVE, 0, s>>>(P, D, tu, tsub, tslot, nt, dnt, task_arcs, sparse, mark, \
                                                        only)
  if (k > 64) {
    if (unit) FL_TASKS(true, 2, 2 * ADS_SB);
    else FL_TASKS(false, 2, 2 * ADS_SB);
  } else if (sb < ADS_SB) {
    if (unit) FL_TASKS(true, 1, ADS_SB / 2);
    else FL_TASKS(false, 1, ADS_SB / 2);
  } else {
    if (unit) FL_TASKS(true, 1, ADS_SB);
    else FL_TASKS(false, 1, ADS_SB);
  }
#undef FL_TASKS
}
static void launch_merge(hipStream_t s, uint32_t grid, bool unit, uint32_t k, uint32_t sb, const AdsArgs &P,
                         uint32_t D, const uint32_t *su, const uint32_t *sfirst, const uint32_t *snt, uint32_t ns,
                         const uint64_t *dns, int mark) {
#define FL_MERGE(U, K, S) \
  k_ads_merge<U, K, S><<<grid, MERGE_WPB * WAVE, 0, s>>>(P, D, su, sfirst, snt, ns, dns, mark)
  if (k > 64) {
    if (unit) FL_MERGE(true, 2, 2 * ADS_SB);
    else FL_MERGE(false, 2, 2 * ADS_SB);
  } else if (sb < ADS_SB) {
    if (unit) FL_MERGE(true, 1, ADS_SB / 2);
    else FL_MERGE(false, 1, ADS_SB / 2);
  } else {
    if (unit) FL_MERGE(true, 1, ADS_SB);
    else FL_MERGE(false, 1, ADS_SB);
  }
#undef FL_MERGE
}

// sb: survivor buffer (ADS_SB / 2 or ads_full_sb(k)).  *buf_over: a level
// overflowed it (the caller restarts with a larger one).
static int ads_run(Ctx &c, const Graph &g, const AdsConfig &cfg, AdsOut &o, bool *need_more, uint32_t sb,
                   bool *buf_over) {
  const uint32_t n = g.n, k = cfg.k, cap = o.cap;
  const uint32_t W = g.w ? g.max_w : 1u;
  const uint32_t NS = W + 1;
  const uint32_t FW = (NS + 31) / 32;
  const bool unit = g.w == nullptr;
  *need_more = false;
  *buf_over = false;

  AdsArgs P{};
  P.n = n;
  P.sb = sb;
  P.k = k;
  P.cap = cap;
  P.W = W;
  P.NS = NS;
  P.FW = FW;
  P.gid = cfg.gid;
  P.seg = cfg.seg;
  P.row_ptr = g.in_ptr;
  P.col = g.in_col;
  P.w = g.in_w;
  P.out_ptr = g.row_ptr;
  P.out_col = g.col;
  P.out_w = g.w;
  P.sk_rank = o.sk_rank;
  P.sk_dist = o.sk_dist;
  P.bk = c.arena->get<uint32_t>((size_t)n * k);
  P.cnt = o.cnt;
  P.lvl = c.arena->get<uint4>((size_t)NS * n);
  P.flags = c.arena->get<uint32_t>((size_t)n * FW);
  P.wl = c.arena->get<uint32_t>((size_t)NS * n);
  P.wl_cnt = c.arena->get<uint32_t>((size_t)NS * CNT_PAD);
  P.ctr = c.arena->get<uint64_t>((size_t)CTR_STRIPES * CTR_FIELDS);
  P.dbg = std::getenv("FL_DEBUG") ? 1u : 0u;
  P.status = c.arena->get<uint32_t>(4);
  P.thr = o.thr;
  P.thr_idx = o.thr ? cfg.thr_idx : nullptr;
  // arc bit planes for the rounds run from worklists (arc positions must fit 32 bits)
  const bool planes = g.m > 0 && g.m < 0xFFFFFFFFull;
  P.plane = nullptr;
  P.pw = g.m / 32 + 2;
  P.out_to_in = nullptr;
  P.flag_from = FLAG_FROM_RINGS * NS;
  P.plane_from = P.flag_from > W ? P.flag_from - W : 0;
  if (planes) {
    P.plane = c.arena->get<uint32_t>((size_t)NS * P.pw);
    fill_u32(c, P.plane, (size_t)NS * P.pw, 0);
    if (g.out_to_in) {
      P.out_to_in = g.out_to_in;
    } else {
      uint32_t *o2i = c.arena->get<uint32_t>(g.m);
      const uint32_t blocks = (uint32_t)std::min<uint64_t>(ceil_div(g.m, 256), 16384);
      k_reverse_arcs<<<blocks, 256, 0, c.s>>>(n, g.m, g.row_ptr, g.col, o2i);
      FL_LAUNCH_CHECK();
      P.out_to_in = o2i;
    }
  }
  fill_u64(c, reinterpret_cast<uint64_t *>(P.lvl), (size_t)NS * n * 2, INF64);  // no level anywhere
  fill_u32(c, P.flags, (size_t)n * FW, 0);
  fill_u32(c, P.wl_cnt, (size_t)NS * CNT_PAD, 0);
  fill_u64(c, P.ctr, (size_t)CTR_STRIPES * CTR_FIELDS, 0);
  fill_u32(c, P.status, 4, 0);

  // scratch slots: enough for every vertex split at once
  {
    uint32_t *need = c.arena->get<uint32_t>(n);
    uint64_t *noff = c.arena->get<uint64_t>((size_t)n + 1);
    k_slot_need<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, g.in_ptr, need);
    FL_LAUNCH_CHECK();
    scan_u32_to_u64(c, need, noff, n);
    FL_HIP(hipMemcpyAsync(c.h_status, noff + n, 8, hipMemcpyDeviceToHost, c.s));
    c.sync();
    const uint64_t slots = c.h_status[0] + 1;
    P.kept = c.arena->get<uint32_t>(slots * sb);
    P.kept_cnt = c.arena->get<uint32_t>(slots);
  }
  // task-list scratch and lists (sized for a list of all vertices)
  const uint64_t max_tasks = (uint64_t)n + g.m / TASK_ARCS + 64;
  TaskScratch ts;
  ts.ntask = c.arena->get<uint32_t>(n);
  ts.nslot = c.arena->get<uint32_t>(n);
  ts.isplit = c.arena->get<uint32_t>(n);
  ts.toff = c.arena->get<uint64_t>((size_t)n + 1);
  ts.soff = c.arena->get<uint64_t>((size_t)n + 1);
  ts.poff = c.arena->get<uint64_t>((size_t)n + 1);
  TaskList tl_dense, tl;
  auto alloc_list = [&](TaskList &t) {
    t.task_u = c.arena->get<uint32_t>(max_tasks);
    t.task_sub = c.arena->get<uint32_t>(max_tasks);
    t.task_slot = c.arena->get<uint32_t>(max_tasks);
    t.split_u = c.arena->get<uint32_t>(n);
    t.split_first = c.arena->get<uint32_t>(n);
    t.split_nt = c.arena->get<uint32_t>(n);
  };
  alloc_list(tl);

  // dense list: vertices with at least one arc, and its static task list
  uint32_t n_dense = 0;
  const bool dense_ok = unit && !(cfg.flags & FL_FLAG_NO_DENSE);
  if (dense_ok) {
    uint32_t *fl = c.arena->get<uint32_t>(n);
    uint64_t *pos = c.arena->get<uint64_t>((size_t)n + 1);
    uint32_t *dense = c.arena->get<uint32_t>(n);
    k_nonisolated_flags<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, g.in_ptr, fl);
    FL_LAUNCH_CHECK();
    scan_u32_to_u64(c, fl, pos, n);
    k_compact<<<(uint32_t)ceil_div(n, 256), 256, 0, c.s>>>(n, fl, pos, dense);
    FL_LAUNCH_CHECK();
    FL_HIP(hipMemcpyAsync(c.h_status, pos + n, 8, hipMemcpyDeviceToHost, c.s));
    c.sync();
    n_dense = (uint32_t)c.h_status[0];
    alloc_list(tl_dense);
    build_tasks(c, g, dense, n_dense, TASK_ARCS, ts, tl_dense);
  }
  // a round marks (so that the next one runs on worklists) once the previous
  // round changed at most a quarter of the dense list
  const uint64_t dense_threshold = (uint64_t)n_dense / 4;

  // round 0
  bool mark = !dense_ok || n_dense <= dense_threshold;
  {
    uint64_t blocks = ceil_div((uint64_t)n * WAVE, 256);
    if (unit) k_ads_init<true><<<(uint32_t)blocks, 256, 0, c.s>>>(P, mark ? 1 : 0);
    else k_ads_init<false><<<(uint32_t)blocks, 256, 0, c.s>>>(P, mark ? 1 : 0);
    FL_LAUNCH_CHECK();
  }
  bool sparse = mark;  // mode of round 1
  hipEvent_t e0 = nullptr, em = nullptr, e1 = nullptr;
  if (c.timing) {
    FL_HIP(hipEventCreate(&e0));
    FL_HIP(hipEventCreate(&em));
    FL_HIP(hipEventCreate(&e1));
  }
  struct EvDel {
    hipEvent_t a, b, c;
    ~EvDel() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (c) (void)hipEventDestroy(c);
    }
  } evdel{e0, em, e1};
  o.kernel_ms = 0.0;
  o.merge_ms = 0.0;
  o.launches = 0;
  uint64_t active_prev = n;
  uint64_t commits_prev = 0;  // commits counted before this round
  std::vector<uint64_t> hctr((size_t)CTR_STRIPES * CTR_FIELDS);
  uint32_t rounds = 0;
  std::vector<uint32_t> hwl(NS);
  bool hwl_valid = false;  // hwl holds the slot counts read back after the previous round
  if (!dense_ok) {
    // Every round runs from worklists.  Rounds are launched RCHUNK at a time
    // with their task lists built on the device (no count goes to the host
    // in between); the round kernels stride over the device-side totals.
    // The host reads back, once per chunk, the work pending after each of
    // its rounds; rounds after the first with nothing pending find empty
    // worklists and change nothing.
    constexpr uint32_t RCHUNK = 16;
    uint64_t *pend = c.arena->get<uint64_t>(2 * RCHUNK);  // [r] pending after round r, [RCHUNK + r] its tasks
    std::vector<hipEvent_t> ev(c.timing ? 3 * RCHUNK : 0, nullptr);
    struct EvVecDel {
      std::vector<hipEvent_t> &v;
      ~EvVecDel() {
        for (hipEvent_t e : v)
          if (e) (void)hipEventDestroy(e);
      }
    } evvd{ev};
    for (auto &e : ev) FL_HIP(hipEventCreate(&e));
    const uint32_t GT = (uint32_t)std::min<uint64_t>(max_tasks, 65536);  // one-wave blocks striding over tasks
    const uint32_t GM = (uint32_t)std::min<uint64_t>(n, 2048);           // merge blocks striding over hubs
    const uint32_t TB = (uint32_t)std::min<uint64_t>(ceil_div(n, 256 * TB_ITEMS), 1024);  // task-list blocks
    const bool pairs = k <= HALF;  // the set of a level fits one half of a wave
    const uint32_t GP = (uint32_t)std::min<uint64_t>(ceil_div(max_tasks, 2), 65536);  // two-task waves
    uint8_t *pend_task = pairs ? c.arena->get<uint8_t>(max_tasks) : nullptr;
    uint64_t *tot = c.arena->get<uint64_t>(3);
    const uint64_t *d_ntasks = tot, *d_nsplit = tot + 2;
    for (uint32_t D0 = 1;; D0 += RCHUNK) {
      for (uint32_t r = 0; r < RCHUNK; ++r) {
        const uint32_t D = D0 + r;
        const uint32_t slot = D % NS;
        const uint32_t task_arcs = (P.plane && D >= P.flag_from) ? TASK_ARCS_FLAGGED : TASK_ARCS_SPARSE;
        fill_u64(c, tot, 3, 0);
        k_task_build<<<TB, 256, 0, c.s>>>(P.wl + (size_t)slot * n, P.wl_cnt + (size_t)slot * CNT_PAD, g.in_ptr, task_arcs, tot,
                                          tl.task_u, tl.task_sub, tl.task_slot, tl.split_u, tl.split_first,
                                          tl.split_nt);
        FL_LAUNCH_CHECK();
        if (c.timing) FL_HIP(hipEventRecord(ev[3 * r], c.s));
        if (pairs) {
          // k <= 32: two small tasks per wave first, then the one-wave kernel on the rest
          if (unit)
            k_ads_pairs<true><<<GP, WAVE, 0, c.s>>>(P, D, tl.task_u, tl.task_sub, tl.task_slot, d_ntasks, pend_task);
          else
            k_ads_pairs<false><<<GP, WAVE, 0, c.s>>>(P, D, tl.task_u, tl.task_sub, tl.task_slot, d_ntasks, pend_task);
          FL_LAUNCH_CHECK();
        }
        launch_tasks(c.s, GT, unit, k, sb, P, D, tl.task_u, tl.task_sub, tl.task_slot, 0, d_ntasks, task_arcs, 1,
                     1, pairs ? pend_task : nullptr);
        FL_LAUNCH_CHECK();
        if (c.timing) FL_HIP(hipEventRecord(ev[3 * r + 1], c.s));
        launch_merge(c.s, GM, unit, k, sb, P, D, tl.split_u, tl.split_first, tl.split_nt, 0, d_nsplit, 1);
        FL_LAUNCH_CHECK();
        if (c.timing) FL_HIP(hipEventRecord(ev[3 * r + 2], c.s));
        fill_u32(c, P.wl_cnt + (size_t)slot * CNT_PAD, 1, 0);
        if (P.plane) fill_u32(c, P.plane + (size_t)slot * P.pw, P.pw, 0);
        k_round_pending<<<1, WAVE, 0, c.s>>>(P.wl_cnt, NS, d_ntasks, pend + r, pend + RCHUNK + r);
        FL_LAUNCH_CHECK();
      }
      std::vector<uint64_t> hp(2 * RCHUNK);
      FL_HIP(hipMemcpyAsync(c.h_status, P.status, 8, hipMemcpyDeviceToHost, c.s));
      FL_HIP(hipMemcpyAsync(hp.data(), pend, 2 * RCHUNK * 8, hipMemcpyDeviceToHost, c.s));
      c.sync();
      const uint32_t st0 = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
      const uint32_t st1 = (uint32_t)(c.h_status[0] >> 32);
      if (st0) {
        *need_more = true;
        return FL_OK;
      }
      if (st1) {
        *buf_over = true;
        return FL_OK;
      }
      uint32_t used = RCHUNK;
      bool done = false;
      for (uint32_t r = 0; r < RCHUNK; ++r)
        if (hp[r] == 0) {
          used = r + 1;
          done = true;
          break;
        }
      // every round of the chunk launched the round kernel (those past the
      // last one with work exit at once): all are counted and timed, as a
      // kernel trace sees them
      for (uint32_t r = 0; r < RCHUNK; ++r) {
        o.launches += 1;
        if (c.timing) {
          float ms = 0.f, ms2 = 0.f;
          FL_HIP(hipEventElapsedTime(&ms, ev[3 * r], ev[3 * r + 1]));
          FL_HIP(hipEventElapsedTime(&ms2, ev[3 * r + 1], ev[3 * r + 2]));
          o.kernel_ms += ms;
          o.merge_ms += ms2;
        }
      }
      rounds = D0 + used - 1;
      if (std::getenv("FL_DEBUG"))
        std::fprintf(stderr, "[fl] rounds %u-%u: tasks of the first %llu, pending after the last %llu\n", D0,
                     D0 + used - 1, (unsigned long long)hp[RCHUNK], (unsigned long long)hp[used - 1]);
      if (done) break;
      // a settled entry is at most (n-1) max_w away: more rounds mean a bug
      if ((uint64_t)D0 + RCHUNK > (uint64_t)(n - 1) * W + 2 + RCHUNK) return FL_EHIP;
    }
  }
  for (uint32_t D = 1; dense_ok; ++D) {
    const uint32_t slot = D % NS;
    const TaskList *T = &tl_dense;
    if (sparse) {
      // slot D is filled by rounds before D, so the previous readback is exact
      uint32_t count = hwl[slot];
      if (!hwl_valid) {
        FL_HIP(hipMemcpyAsync(c.h_status, P.wl_cnt + (size_t)slot * CNT_PAD, 4, hipMemcpyDeviceToHost, c.s));
        c.sync();
        count = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
      }
      build_tasks(c, g, P.wl + (size_t)slot * n, count,
                  (P.plane && D >= P.flag_from) ? TASK_ARCS_FLAGGED : TASK_ARCS_SPARSE, ts, tl);
      T = &tl;
    }
    // marking decision for this round (decides the mode of the next one)
    mark = !dense_ok || active_prev <= dense_threshold;
    if (T->ntasks) {
      if (c.timing) FL_HIP(hipEventRecord(e0, c.s));
      const uint32_t tb = (uint32_t)ceil_div(T->ntasks, TASK_WPB);
      launch_tasks(c.s, tb, unit, k, sb, P, D, T->task_u, T->task_sub, T->task_slot, T->ntasks, nullptr,
                   T->task_arcs, sparse ? 1 : 0, mark ? 1 : 0);
      FL_LAUNCH_CHECK();
      if (c.timing) FL_HIP(hipEventRecord(em, c.s));
      if (T->nsplit) {
        const uint32_t mb = T->nsplit;  // one block of MERGE_WPB waves per split vertex
        launch_merge(c.s, mb, unit, k, sb, P, D, T->split_u, T->split_first, T->split_nt, T->nsplit, nullptr,
                     mark ? 1 : 0);
        FL_LAUNCH_CHECK();
      }
      if (c.timing) FL_HIP(hipEventRecord(e1, c.s));
    }
    if (sparse) fill_u32(c, P.wl_cnt + (size_t)slot * CNT_PAD, 1, 0);
    // the plane of this round is read; commits of later rounds refill it
    if (P.plane) fill_u32(c, P.plane + (size_t)slot * P.pw, P.pw, 0);
    ++rounds;
    FL_HIP(hipMemcpyAsync(c.h_status, P.status, 8, hipMemcpyDeviceToHost, c.s));
    FL_HIP(hipMemcpyAsync(hctr.data(), P.ctr, hctr.size() * 8, hipMemcpyDeviceToHost, c.s));
    fetch_padded(c, hwl.data(), P.wl_cnt, NS);  // waits for both
    hwl_valid = true;
    if (T->ntasks) {
      float ms = 0.f, ms2 = 0.f;
      if (c.timing) {
        FL_HIP(hipEventElapsedTime(&ms, e0, em));
        FL_HIP(hipEventElapsedTime(&ms2, em, e1));
      }
      o.kernel_ms += ms;
      o.merge_ms += ms2;
      o.launches += 1;
      if (std::getenv("FL_DEBUG")) {
        std::vector<uint64_t> hs((size_t)CTR_STRIPES * CTR_FIELDS), f(CF_COUNT, 0);
        FL_HIP(hipMemcpy(hs.data(), P.ctr, hs.size() * 8, hipMemcpyDeviceToHost));
        for (uint32_t i = 0; i < CTR_STRIPES; ++i)
          for (uint32_t q = 0; q < CF_COUNT; ++q) f[q] += hs[(size_t)i * CTR_FIELDS + q];
        const uint64_t ex = f[CF_EXAMINED], sv = f[CF_SURVIVORS], pr = f[CF_PRUNES], sc = f[CF_SCANNED],
                       mt = f[CF_MATCHED], ma = f[CF_MARK_ARCS], mp = f[CF_MARKED];
        const uint64_t act = f[CF_COMMITS] - commits_prev;
        std::fprintf(stderr, "[fl] round %u: %s, %u tasks, %u split, %llu changed, %.2f ms, merge %.2f ms, "
                     "examined(cum) %.3fG survivors(cum) %.3fG prunes(cum) %.3fM scanned(cum) %.3fG "
                     "matched(cum) %.3fG markarcs(cum) %.3fG marked(cum) %.3fG\n",
                     D, sparse ? "sparse" : "dense", T->ntasks, T->nsplit, (unsigned long long)act, ms, ms2,
                     ex / 1e9, sv / 1e9, pr / 1e6, sc / 1e9, mt / 1e9, ma / 1e9, mp / 1e9);
      }
    }
    const uint32_t st0 = (uint32_t)(c.h_status[0] & 0xFFFFFFFFu);
    const uint32_t st1 = (uint32_t)(c.h_status[0] >> 32);
    if (st0) {
      *need_more = true;
      return FL_OK;
    }
    if (st1) {
      *buf_over = true;
      return FL_OK;
    }
    uint64_t commits = 0;
    for (uint32_t i = 0; i < CTR_STRIPES; ++i) commits += hctr[(size_t)i * CTR_FIELDS + CF_COMMITS];
    const uint64_t active = commits - commits_prev;  // vertices that changed this round
    commits_prev = commits;
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
  std::vector<uint64_t> hc((size_t)CTR_STRIPES * CTR_FIELDS);
  FL_HIP(hipMemcpyAsync(hc.data(), P.ctr, hc.size() * 8, hipMemcpyDeviceToHost, c.s));
  c.sync();
  o.relax_exec = 0;
  for (uint32_t i = 0; i < CTR_STRIPES; ++i) o.relax_exec += hc[(size_t)i * CTR_FIELDS + CF_EXAMINED];
  return FL_OK;
}

int ads_build(Ctx &c, const Graph &g, const AdsConfig &cfg, AdsOut &o) {
  if (cfg.k == 0) return FL_EINVAL;
  if (cfg.k > MAX_K) return FL_ENOTIMPL;
  if (g.w && g.max_w > MAX_W) return FL_ENOTIMPL;
  if (!g.in_ptr) return FL_EINVAL;  // the in-arc view is set by set_in_arcs
  uint32_t cap = ads_capacity(cfg.n_cap ? cfg.n_cap : g.n, cfg.k);
  // half the survivor buffer for k <= 32 (FL_TEST_SMALL_SURVIVOR_BUFFER: for
  // k <= 64 too, so that tests reach the restart below on small graphs)
  const uint32_t small_k = std::getenv("FL_TEST_SMALL_SURVIVOR_BUFFER") ? 64u : 32u;
  uint32_t sb = cfg.k <= small_k ? ADS_SB / 2 : ads_full_sb(cfg.k);
  for (int attempt = 0; attempt < 7; ++attempt) {
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
    bool more = false, buf_over = false;
    int rc = ads_run(c, g, cfg, o, &more, sb, &buf_over);
    if (rc != FL_OK) return rc;
    c.arena->rewind(after_out);
    if (buf_over) {
      // a level overflowed the survivor buffer: again with the full one
      if (sb >= ads_full_sb(cfg.k)) return FL_ENOMEM;
      if (std::getenv("FL_DEBUG")) std::fprintf(stderr, "[fl] sketches: survivor buffer %u overflowed\n", sb);
      sb = ads_full_sb(cfg.k);
      c.arena->rewind(mark);
      continue;
    }
    if (std::getenv("FL_DEBUG"))
      std::fprintf(stderr, "[fl] sketches: cap %u rounds %u overflow %d\n", cap, o.rounds, (int)more);
    if (!more) {
      // rows without a threshold row keep rank order within a level: only
      // the rows of facilities (every row for fl_ads_build) are read later
      if (o.thr && thr_rows) {
        const uint32_t tgrid = (uint32_t)ceil_div((uint64_t)thr_rows * WAVE, 256);
        if (cfg.k <= 64)
          k_hip_thresholds<1><<<tgrid, 256, 0, c.s>>>(thr_rows, cfg.thr_rows_vertex, cap, cfg.k, o.cnt, o.sk_rank, o.thr);
        else
          k_hip_thresholds<2><<<tgrid, 256, 0, c.s>>>(thr_rows, cfg.thr_rows_vertex, cap, cfg.k, o.cnt, o.sk_rank, o.thr);
        FL_LAUNCH_CHECK();
      }
      return FL_OK;
    }
    uint64_t nc = (uint64_t)cap * 3 / 2 + 16;
    const uint32_t nmax = cfg.n_cap ? cfg.n_cap : g.n;
    if (nc > nmax) nc = nmax;
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
