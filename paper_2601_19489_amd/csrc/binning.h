// The run tables that the binning leaves in its workspace, for the forward
// that writes the tile lists itself as it reaches them (the deferred form of
// the binning: identical lists, but only the positions the compositing
// reaches are written).
#pragma once

#include "common.h"

namespace gs {

constexpr int kSegSlots = 8;                 // runs per lane of a segment's wavefront
constexpr int kSegRuns = kWave * kSegSlots;  // runs per segment

struct RunLists {
  const uint2* runs;         // (Gaussian id, first row | length << 16), by column, depth order
  const uint32_t* cstart;    // [tiles_x + 1] first run of each column
  const uint32_t* segfirst;  // [tiles_x + 1] first segment of each column
  const uint32_t* hist;      // [segment][tiles_y] list position of the segment's first entry
};

// The tables inside a binning workspace of at least the size the binning
// needs for (n, cap) and the tile grid; false if `bytes` is smaller.
bool run_lists(const void* workspace, size_t bytes, int64_t n, int64_t cap, int tiles_x,
               int tiles_y, RunLists* out);

}  // namespace gs
