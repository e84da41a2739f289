// fl_ads.h -- sketch construction interface (internal).
#pragma once
#include "fl_common.h"

namespace fl {

struct AdsConfig {
  uint32_t k;
  const uint32_t *gid;       // [n] graph of each vertex of a union (nullptr: one graph)
  const SegInfo *seg;        // device table of the graphs (keys, base, bucket shift)
  uint32_t flags;
  uint32_t thr_rows;         // rows of the HIP-threshold table (0 = none)
  const uint32_t *thr_idx;   // [n] row of each vertex (INF32 = none); nullptr = row u
  const uint32_t *thr_rows_vertex;  // [thr_rows] vertex of each row; nullptr = row r is vertex r
  uint32_t n_cap;            // vertex count of the largest graph (sizes the rows)
};

struct AdsOut {
  uint32_t cap = 0;          // per-vertex capacity (entries)
  uint32_t *sk_rank = nullptr;  // [n * cap]
  uint32_t *sk_dist = nullptr;  // [n * cap]
  uint32_t *cnt = nullptr;      // [n] entries per vertex
  uint32_t *thr = nullptr;      // [thr_rows * cap] HIP thresholds (0 = 2^32)
  const uint32_t *thr_idx = nullptr;
  uint32_t rounds = 0;
  uint64_t relax_exec = 0;
  double kernel_ms = 0.0;     // summed device time of the round-kernel (k_ads_tasks) launches
  double merge_ms = 0.0;      // summed device time of the split-vertex merge launches
  uint32_t launches = 0;
};

uint32_t ads_capacity(uint32_t n, uint32_t k);
// device bytes the construction needs besides its outputs
size_t ads_scratch_bytes(uint32_t n, uint64_t m, uint32_t k, uint32_t NS);
int ads_build(Ctx &c, const Graph &g, const AdsConfig &cfg, AdsOut &o);
int ads_export(Ctx &c, const Graph &g, const AdsOut &o, uint64_t *off, uint32_t *rank, uint32_t *dist,
               uint32_t *thr);

}  // namespace fl
