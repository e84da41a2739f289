// fl_mis.h -- facility selection interface (internal).
#pragma once
#include <vector>

#include "fl_common.h"

namespace fl {

struct MisIn {
  const Graph *g;
  uint32_t G;                       // graphs in the union
  const uint32_t *gid;              // [n] graph of each vertex (nullptr when G == 1)
  const SegInfo *seg;               // [G] device (priority keys)
  std::vector<uint32_t> rungs;      // per graph: rungs of the opening loop
  const std::vector<std::vector<double>> *lad;  // per graph ladder
  double eps;
  const uint32_t *orung;  // [n]
  const uint32_t *frz;    // [n]
  bool luby;              // Luby's variant: priorities redrawn every round
};

// rounds_out[g]: MIS rounds of graph g, summed over its rungs
int mis_phase(Ctx &c, const MisIn &in, uint8_t *open, std::vector<uint32_t> &rounds_out);

}  // namespace fl
