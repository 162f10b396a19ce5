// tune.hpp -- autotuner table of the elimination schedules.
//
// A level is eliminated by one of several schedules that give the same
// factor up to rounding:
//   kSchedPersistent  one cooperative launch for all colours of the level
//                     (one workgroup per cluster, grid barrier between
//                     colours); `grid_cap` > 0 limits the resident grid
//   kSchedPerColour   one launch per colour, one workgroup per cluster
//   kSchedSplit       per colour, one launch per elimination step with
//                     several workgroups per cluster (96..512 DoFs); `tile`
//                     picks the column tile of the scaling step
// The tuner times the candidates on the level itself and records the
// fastest under a key made of the level's shape.  The table persists as a
// small JSON file (lrsp_autotune_save / lrsp_autotune_load).
#pragma once
#include <cstdint>
#include <string>

#include "../../include/lrsp.h"

namespace lrsp {
namespace tune {

enum Sched { kSchedPersistent = 0, kSchedPerColour = 1, kSchedSplit = 2 };

struct Choice {
  int sched = kSchedPersistent;
  int grid_cap = 0;
  double ms = 0.0;
  int tile = 0;  // kSchedSplit: column tile of the scaling step (kTileWide / kTileNarrow)
};

// Key of a level: batched or not, largest cluster (rounded up to 32),
// clusters (rounded up to a power of two) and colours.
std::string key(bool batched, int max_m, int nitems, int ncolours);
bool lookup(const std::string& k, Choice* c);
void store(const std::string& k, const Choice& c);
int entries();
void clear();
lrsp_status save(const char* path);
lrsp_status load(const char* path);

}  // namespace tune
}  // namespace lrsp
