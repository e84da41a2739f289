// fl_mis.h -- facility selection interface (internal).
#pragma once
#include <vector>

#include "fl_common.h"

namespace fl {

struct MisIn {
  const Graph *g;
  uint32_t rungs;
  const std::vector<double> *lad;
  double eps;
  const uint32_t *orung;  // [n]
  const uint32_t *frz;    // [n]
  PermKey pk;             // priority key
};

int mis_phase(Ctx &c, const MisIn &in, uint8_t *open, uint32_t *rounds_out);

}  // namespace fl
