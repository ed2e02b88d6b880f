// Tuning constants of the instance binning (expansion and per-tile counters).
// Kept apart from the headers of the compositing kernels, which they do not affect.
#pragma once

#include "gps_internal.h"

namespace gps {

constexpr int kExpG = 64;             // view-Gaussians per block of the instance expansion (kBlk lanes walk
                                      // their tile rectangles: about kBlk / kExpG lanes per Gaussian)
constexpr int kExpGLog2 = 6;
static_assert((1 << kExpGLog2) == kExpG && kBlk % kExpG == 0, "expansion share");
constexpr int kCntSplit = 4;          // sub-counters per tile for the count pass's atomics (block index mod 4):
                                      // fewer increments queue on one address
constexpr int kSmallSort = 512;       // one wavefront sorts up to this many keys in registers
// Tiles of at least kLongTile keys (exactly those whose queue bucket floor(log2(n + 1))
// is log2(kSmallSort) or more, so they lead the longest-first queue) take the block sort.
constexpr unsigned int kLongTile = kSmallSort - 1;

}  // namespace gps
