// fl_frontier.h -- long rows of a frontier, cut into pieces.  A frontier
// kernel flattens short rows over the wave (flat_arcs) and queues each long
// row as pieces of HCHUNK arcs; a second kernel walks the queue with one wave
// per piece, so the arcs of a hub are spread over many waves.
#pragma once

#include "fl_common.h"

namespace fl {

// arcs per queued piece: hubs split finely enough to keep the long-row
// kernels' waves busy (MIS 0.935 -> 0.907 s on the large weighted workload
// against 2,048-arc pieces, timed on one box, identical results)
constexpr uint32_t HCHUNK = 512;
// blocks (of 256 threads) of a long-row kernel: it walks a device-side count
// with one wave per piece, so it needs many waves per CU to hide the random
// accesses of hub rows (16 per CU on 256 CUs); idle blocks exit at once
constexpr uint32_t HEAVY_BLOCKS = 1024;

// queue entries needed for n vertices and m arcs at most
inline uint64_t piece_capacity(uint64_t n, uint64_t m) { return n + m / HCHUNK + 64; }

// Every lane calls.  Lanes with heavy == true queue their row as pieces:
// entry = piece << 32 | vertex.
__device__ inline void push_pieces(uint64_t *q, uint32_t *qcnt, bool heavy, uint32_t x, uint64_t deg) {
  const uint32_t np = heavy ? (uint32_t)((deg + HCHUNK - 1) / HCHUNK) : 0u;
  const uint32_t incl = wave_scan_incl(np);
  const uint32_t tot = __shfl(incl, WAVE - 1, WAVE);
  if (!tot) return;
  uint32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(qcnt, tot);
  base = __shfl(base, 0, WAVE);
  for (uint32_t p = 0; p < np; ++p) q[base + incl - np + p] = ((uint64_t)p << 32) | x;
}

// arcs [*b0, *b1) of queue entry e
__device__ inline uint32_t piece_arcs(uint64_t e, const uint64_t *row_ptr, uint64_t *b0, uint64_t *b1) {
  const uint32_t x = (uint32_t)e;
  const uint64_t p = e >> 32;
  const uint64_t a0 = row_ptr[x], a1 = row_ptr[x + 1];
  *b0 = a0 + p * HCHUNK;
  *b1 = *b0 + HCHUNK < a1 ? *b0 + HCHUNK : a1;
  return x;
}

}  // namespace fl
