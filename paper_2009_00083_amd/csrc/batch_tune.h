// Batch launch configuration: how many fields share a launch and how many
// wave tiles each field aims at, set by the caller or by the autotuner.
#pragma once

#include <stdint.h>

#include "pcrit_internal.h"

namespace pcrit {

// Tile planning with an explicit target number of wave tiles: the deepest
// tile (a multiple of the kernel's unroll, up to its staging cap) that still
// gives `want` tiles.
void plan_level3_want(LevelDesc &l, bool write_masks, int64_t want);
void plan_level2_want(LevelDesc &l, int64_t want);

constexpr int kBatchGroupDefault = kMaxFused;  // fields per shared launch
// Wave tiles per field.  Measured on 200 fields of 33..257 samples per axis
// (16 fields per launch): 128, 256 and 512 tiles 1.91 ms, 1024 1.94, 2048
// 2.06, 4096 2.33 ms; fewer tiles keep the fused kernel's full-depth tiles.
constexpr int64_t kBatchWantDefault = 512;
constexpr int64_t kBatchWantMin = 64, kBatchWantMax = 1 << 20;

}  // namespace pcrit
