// Step 1 of localized topological simplification on the GPU (gfx950): the
// superlevel (sublevel) set propagation from every maximum (minimum) of the
// order field, Section 4.2, with the persistence test of Section 4.5.
//
// One thread per extremum.  The thread grows the extremum's component one
// vertex at a time, always taking the largest vertex (in the order field,
// reversed for minima) adjacent to it, and stops when the vertex just taken
//   - lies more than epsilon in value from the extremum: persistent;
//   - has a larger neighbour outside the component: that vertex is the
//     saddle where the component meets another one;
// or when the component holds max_visited vertices or more than
// max_frontier vertices wait outside it (budget).  Component and waiting
// vertices live in per-thread arrays (private memory); membership is a
// linear scan, which stays cheap for the small components that noise
// extrema have.  The propagations are independent: merging propagations
// that meet at a saddle (hill chains) is not done here.
#include <stdint.h>

#include "pcrit_internal.h"
#include "lts.h"

namespace pcrit {
namespace {

// Freudenthal neighbour offsets (dx, dy, dz): the positive ones, then
// their negatives; 2D uses the first three and their negatives.
__constant__ int8_t kNb3[14][3] = {{1, 0, 0},   {0, 1, 0},   {1, 1, 0},   {0, 0, 1},   {1, 0, 1},
                                   {0, 1, 1},   {1, 1, 1},   {-1, 0, 0},  {0, -1, 0},  {-1, -1, 0},
                                   {0, 0, -1},  {-1, 0, -1}, {0, -1, -1}, {-1, -1, -1}};
__constant__ int8_t kNb2[6][3] = {{1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {-1, -1, 0}};

struct Grid {
  int64_t nx, ny, nz, n;
};

// Neighbour k of vertex v (x, y, z), or -1 outside the grid.
template <int DIM>
__device__ __forceinline__ int64_t neighbour(const Grid &g, int64_t x, int64_t y, int64_t z,
                                             int k) {
  const int8_t *o = DIM == 3 ? kNb3[k] : kNb2[k];
  const int64_t a = x + o[0], b = y + o[1], c = z + o[2];
  if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) return -1;
  return (c * g.ny + b) * g.nx + a;
}

template <int DIM>
__global__ __launch_bounds__(256) void lts_propagate_kernel(
    const float *f, const uint32_t *rank, Grid g, const uint32_t *ext, int64_t n_ext,
    uint32_t flip, float eps, int max_visited, int max_frontier, uint8_t *status,
    int32_t *saddle, uint16_t *visited) {
  constexpr int NB = DIM == 3 ? 14 : 6;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ext) return;
  const int64_t m = ext[i];
  if (m < 0 || m >= g.n) {  // not a vertex of the grid
    status[i] = kLtsInvalid;
    saddle[i] = -1;
    visited[i] = 0;
    return;
  }
  const bool maxima = flip == 0u;
  uint32_t comp[kLtsMaxVisited];
  uint32_t wv[kLtsMaxFrontier + 14], wk[kLtsMaxFrontier + 14];
  int nc = 1, nw = 0;
  comp[0] = (uint32_t)m;
  const float fm = f[m];
  auto key = [&](int64_t u) { return rank[u] ^ flip; };
  auto in_comp = [&](uint32_t u) {
    for (int j = 0; j < nc; j++)
      if (comp[j] == u) return true;
    return false;
  };
  auto waiting = [&](uint32_t u) {
    for (int j = 0; j < nw; j++)
      if (wv[j] == u) return true;
    return false;
  };
  {
    const int64_t x = m % g.nx, y = (m / g.nx) % g.ny, z = m / (g.nx * g.ny);
    for (int k = 0; k < NB; k++) {
      const int64_t u = neighbour<DIM>(g, x, y, z, k);
      if (u < 0) continue;
      wv[nw] = (uint32_t)u;
      wk[nw] = key(u);
      nw++;
    }
  }
  uint8_t st = kLtsBudget;
  int32_t sd = -1;
  while (nw > 0) {
    // take the largest waiting vertex
    int b = 0;
    for (int j = 1; j < nw; j++)
      if (wk[j] > wk[b]) b = j;
    const uint32_t v = wv[b], kv = wk[b];
    wv[b] = wv[nw - 1];
    wk[b] = wk[nw - 1];
    nw--;
    comp[nc++] = v;
    const float d = maxima ? fm - f[v] : f[v] - fm;
    if (d > eps) {
      st = kLtsPersistent;
      break;
    }
    const int64_t x = v % g.nx, y = (v / g.nx) % g.ny, z = v / (g.nx * g.ny);
    bool is_saddle = false;
    for (int k = 0; k < NB && !is_saddle; k++) {
      const int64_t u = neighbour<DIM>(g, x, y, z, k);
      if (u >= 0 && key(u) > kv && !in_comp((uint32_t)u)) is_saddle = true;
    }
    if (is_saddle) {
      st = kLtsSaddle;
      sd = (int32_t)v;
      break;
    }
    if (nc >= max_visited) break;
    for (int k = 0; k < NB; k++) {
      const int64_t u = neighbour<DIM>(g, x, y, z, k);
      if (u < 0 || in_comp((uint32_t)u) || waiting((uint32_t)u)) continue;
      wv[nw] = (uint32_t)u;
      wk[nw] = key(u);
      nw++;
    }
    if (nw > max_frontier) break;
  }
  status[i] = st;
  saddle[i] = sd;
  visited[i] = (uint16_t)nc;
}

}  // namespace

hipError_t launch_lts_propagate(const float *f, const uint32_t *rank, int64_t nx, int64_t ny,
                                int64_t nz, const uint32_t *ext, int64_t n_ext, bool maxima,
                                float eps, int max_visited, int max_frontier, uint8_t *status,
                                int32_t *saddle, uint16_t *visited, hipStream_t st) {
  if (n_ext == 0) return hipSuccess;
  if (max_visited < 2 || max_visited > kLtsMaxVisited || max_frontier < 14 ||
      max_frontier > kLtsMaxFrontier)
    return hipErrorInvalidValue;
  const Grid g{nx, ny, nz, nx * ny * nz};
  const dim3 grid((unsigned)((n_ext + 255) / 256)), block(256);
  const uint32_t flip = maxima ? 0u : 0xFFFFFFFFu;
  if (nz > 1)
    hipLaunchKernelGGL(lts_propagate_kernel<3>, grid, block, 0, st, f, rank, g, ext, n_ext, flip,
                       eps, max_visited, max_frontier, status, saddle, visited);
  else
    hipLaunchKernelGGL(lts_propagate_kernel<2>, grid, block, 0, st, f, rank, g, ext, n_ext, flip,
                       eps, max_visited, max_frontier, status, saddle, visited);
  return hipGetLastError();
}

}  // namespace pcrit
