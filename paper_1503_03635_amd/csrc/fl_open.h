// fl_open.h -- opening loop interface (internal).
#pragma once
#include <vector>

#include "fl_ads.h"
#include "fl_common.h"

namespace fl {

struct OpenIn {
  const Graph *g;
  uint32_t nF;
  const uint32_t *fac_list;  // [nF] facility vertex ids, increasing
  const uint32_t *fac_idx;   // [n] facility index or INF32
  const uint32_t *fac_cost;  // [n]
  const AdsOut *ads;         // thr rows by facility index
  PermKey rk;
  const uint8_t *ceff;       // [n] served clients (reach a facility)
  uint64_t nCeff;
  uint64_t nUF0;             // facilities that are served clients
  const uint64_t *gam_lab;   // [n] (gamma_c << 32 | minimising facility)
  double eps;
  std::vector<double> *lad;  // ladder a[0..], grown on demand
};

struct OpenOut {
  uint32_t *orung;  // [n]
  uint32_t *frz;    // [n]
  double *q;        // [nF]
  uint32_t rungs = 0;
  uint32_t nO = 0;
};

int open_phase(Ctx &c, const OpenIn &in, OpenOut &out);

}  // namespace fl
