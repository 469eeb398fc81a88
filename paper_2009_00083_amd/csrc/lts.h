// LTS Step 1 on the GPU: the launcher the C ABI calls and its limits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcrit {

// LTS Step 1: the superlevel (maxima) or sublevel (minima) set propagation
// from each extremum ext[0 .. n_ext) of a grid with order field `rank`;
// per extremum a status (kLts*), the saddle (or -1) and the vertices taken.
constexpr int kLtsMaxVisited = 32;    // largest max_visited
constexpr int kLtsMaxFrontier = 128;  // largest max_frontier
constexpr uint8_t kLtsSaddle = 0, kLtsPersistent = 1, kLtsBudget = 2, kLtsInvalid = 3;
// Merged propagations (propagations that meet at a saddle continue as one,
// led by the largest extremum): the same outputs per listed extremum, with
// scratch of lts_merged_scratch_bytes(n_ext) bytes; at most kLtsMaxMerged
// extrema per launch.
constexpr int64_t kLtsMaxMerged = int64_t(1) << 30;
size_t lts_merged_scratch_bytes(int64_t n_ext);
hipError_t launch_lts_merged(const float *f, const uint32_t *rank, int64_t nx, int64_t ny,
                             int64_t nz, const uint32_t *ext, int64_t n_ext, bool maxima,
                             float eps, int max_visited, int max_frontier, uint8_t *status,
                             int32_t *saddle, uint16_t *visited, void *scratch, hipStream_t st);
hipError_t launch_lts_propagate(const float *f, const uint32_t *rank, int64_t nx, int64_t ny,
                                int64_t nz, const uint32_t *ext, int64_t n_ext, bool maxima,
                                float eps, int max_visited, int max_frontier, uint8_t *status,
                                int32_t *saddle, uint16_t *visited, hipStream_t st);

}  // namespace pcrit
