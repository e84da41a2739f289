// fl_open.h -- opening loop interface (internal).
#pragma once
#include <vector>

#include "fl_ads.h"
#include "fl_common.h"

namespace fl {

struct OpenIn {
  const Graph *g;
  uint32_t G;                // graphs in the union
  const uint32_t *gid;       // [n] graph of each vertex (nullptr when G == 1)
  const SegInfo *seg;        // [G] device
  uint32_t nF;
  const uint32_t *fac_list;  // [nF] facility vertex ids, increasing
  const uint32_t *fac_idx;   // [n] facility index or INF32
  const uint32_t *fac_cost;  // [n]
  const AdsOut *ads;         // thr rows by facility index
  const uint8_t *ceff;       // [n] served clients (reach a facility)
  std::vector<uint64_t> nF_g;   // per graph: facilities
  std::vector<uint64_t> nCeff;  // per graph: served clients
  std::vector<uint64_t> nUF0;   // per graph: facilities that are served clients
  const uint64_t *gam_lab;   // [n] (gamma_c << 32 | minimising facility)
  double eps;
  std::vector<std::vector<double>> *lad;  // per graph ladder a[0..], grown on demand
};

struct OpenOut {
  uint32_t *orung;  // [n]
  uint32_t *frz;    // [n]
  double *q;        // [nF]
  std::vector<uint32_t> rungs;  // per graph
  std::vector<uint64_t> nO;     // per graph
  std::vector<int> rc;          // per graph (FL_ERANGE if the ladder overflows)
};

int open_phase(Ctx &c, const OpenIn &in, OpenOut &out);

}  // namespace fl
