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

#include <algorithm>

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
    // The vertices are taken in decreasing order (a larger vertex next to
    // the component would have made the previous one a saddle), so every
    // vertex of the component but v is larger than v: a smaller neighbour
    // of v is outside it, and a larger one is inside unless v is a saddle.
    const int64_t x = v % g.nx, y = (v / g.nx) % g.ny, z = v / (g.nx * g.ny);
    int64_t nu[NB];
    uint32_t nk[NB];
#pragma unroll
    for (int k = 0; k < NB; k++) {
      nu[k] = neighbour<DIM>(g, x, y, z, k);
      nk[k] = nu[k] >= 0 ? key(nu[k]) : 0u;
    }
    bool is_saddle = false;
#pragma unroll
    for (int k = 0; k < NB; k++)
      if (!is_saddle && nu[k] >= 0 && nk[k] > kv && !in_comp((uint32_t)nu[k])) is_saddle = true;
    if (is_saddle) {
      st = kLtsSaddle;
      sd = (int32_t)v;
      break;
    }
    if (nc >= max_visited) break;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] < 0 || nk[k] > kv || waiting((uint32_t)nu[k])) continue;
      wv[nw] = (uint32_t)nu[k];
      wk[nw] = nk[k];
      nw++;
    }
    if (nw > max_frontier) break;
  }
  status[i] = st;
  saddle[i] = sd;
  visited[i] = (uint16_t)nc;
}

// Merged propagations (Sections 4.4 and 4.5).  Scratch: one record per
// listed extremum (its component, its waiting vertices, its leader, the
// next record parked at the same saddle) and an open-addressing table of
// saddles (vertex, higher neighbours taken by the arrivals so far, the last
// record parked there).
constexpr int kRecWords = 4 + kLtsMaxVisited + kLtsMaxFrontier;
constexpr uint32_t kNone = 0xFFFFFFFFu;
// arrivals at one saddle: each holds one of its (at most 14) higher neighbours
constexpr uint32_t kMaxArrivals = 16;

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  // integer hash "lowbias32" (C. Wellons, hash-prospector)
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return h;
}

__global__ __launch_bounds__(256) void lts_table_clear_kernel(uint32_t *tkey, uint32_t *tcnt,
                                                              uint32_t *thead, uint32_t cap) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cap; j += gridDim.x * blockDim.x) {
    tkey[j] = kNone;
    tcnt[j] = 0;
    thead[j] = kNone;
  }
}

// One thread per listed extremum.  The propagation grows as in
// lts_propagate_kernel, led by the extremum, until it stops at a saddle s.
// There it parks its state in its record, joins s's list and adds the
// higher neighbours of s it holds to s's count; the thread whose addition
// completes the count (all higher neighbours of s taken) takes over every
// parked state, keeps the largest leader and goes on from s.  The other
// leaders keep the saddle status written at their arrival.  No thread
// waits for another, so every thread ends after at most max_visited takes
// and merges.
template <int DIM>
__global__ __launch_bounds__(256) void lts_merge_kernel(
    const float *f, const uint32_t *rank, Grid g, const uint32_t *ext, int64_t n_ext,
    uint32_t flip, float eps, int max_visited, int max_frontier, uint8_t *status,
    int32_t *saddle, uint16_t *visited, uint32_t *rec, uint32_t *tkey, uint32_t *tcnt,
    uint32_t *thead, uint32_t tmask) {
  constexpr int NB = DIM == 3 ? 14 : 6;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ext) return;
  auto key = [&](int64_t u) { return rank[u] ^ flip; };
  const int64_t m = ext[i];
  bool ok = m < g.n;
  if (ok) {  // an extremum of the kind asked for: every neighbour earlier in the order
    const int64_t x = m % g.nx, y = (m / g.nx) % g.ny, z = m / (g.nx * g.ny);
    const uint32_t km = key(m);
    for (int k = 0; k < NB; k++) {
      const int64_t u = neighbour<DIM>(g, x, y, z, k);
      if (u >= 0 && key(u) > km) ok = false;
    }
  }
  if (!ok) {
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
  uint32_t lead = (uint32_t)i;
  float fl = f[m];
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
  uint8_t st;
  for (;;) {
    if (nw == 0) {  // the whole grid taken: nothing ends this extremum
      st = kLtsPersistent;
      break;
    }
    int b = 0;
    for (int j = 1; j < nw; j++)
      if (wk[j] > wk[b]) b = j;
    const uint32_t v = wv[b], kv = wk[b];
    wv[b] = wv[nw - 1];
    wk[b] = wk[nw - 1];
    nw--;
    comp[nc++] = v;
    const float d = maxima ? fl - f[v] : f[v] - fl;
    if (d > eps) {
      st = kLtsPersistent;
      break;
    }
    // taken in decreasing order (merges keep it: a merged component holds
    // the vertices above the saddle, everything waiting lies below), so a
    // smaller neighbour of v is outside the component
    const int64_t x = v % g.nx, y = (v / g.nx) % g.ny, z = v / (g.nx * g.ny);
    int64_t nu[NB];
    uint32_t nk[NB];
#pragma unroll
    for (int k = 0; k < NB; k++) {
      nu[k] = neighbour<DIM>(g, x, y, z, k);
      nk[k] = nu[k] >= 0 ? key(nu[k]) : 0u;
    }
    uint32_t nh = 0, mine = 0;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] >= 0 && nk[k] > kv) {
        nh++;
        mine += in_comp((uint32_t)nu[k]) ? 1u : 0u;
      }
    }
    if (mine < nh) {
      // arrival at the saddle v: park, join v's list, add to its count
      uint32_t *r = rec + (size_t)i * kRecWords;
      r[0] = (uint32_t)nc;
      r[1] = (uint32_t)nw;
      r[2] = lead;
      for (int j = 0; j < nc; j++) r[4 + j] = comp[j];
      for (int j = 0; j < nw; j++) r[4 + kLtsMaxVisited + j] = wv[j];
      status[lead] = kLtsSaddle;
      saddle[lead] = (int32_t)v;
      visited[lead] = (uint16_t)nc;
      uint32_t h = mix32(v) & tmask;
      for (uint32_t probe = 0; probe <= tmask; probe++) {  // at most half full: ends
        const uint32_t k = atomicCAS(&tkey[h], kNone, v);
        if (k == kNone || k == v) break;
        h = (h + 1) & tmask;
      }
      r[3] = atomicExch(&thead[h], (uint32_t)i);
      // release: the record, the list link and the leader's provisional
      // status reach every XCD before the count does; acquire (last arrival
      // only): the records parked by the others are read after the count.
      // A full fence on every arrival would also drop the L2 lines of the
      // field and the order field that the other propagations are reading.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint32_t before = atomicAdd(&tcnt[h], mine);
      if (before + mine != nh) return;  // not the last arrival
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // the last arrival: the largest leader leads the union
      const uint32_t head = __hip_atomic_load(&thead[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int total = nc;
      uint32_t best = lead, bkey = key(ext[lead]);
      // every record in the list was written by an arrival of this launch:
      // index, counts and leader are in range (the checks only keep a
      // broken invariant from reading past the buffers)
      for (uint32_t q = head, step = 0; q < (uint32_t)n_ext && step < kMaxArrivals;
           q = rec[(size_t)q * kRecWords + 3], step++) {
        if (q == (uint32_t)i) continue;
        const uint32_t *o = rec + (size_t)q * kRecWords;
        total += (int)min(o[0], (uint32_t)kLtsMaxVisited) - 1;  // v is in every parked component
        const uint32_t ol = min(o[2], (uint32_t)(n_ext - 1));
        const uint32_t kl = key(ext[ol]);
        if (kl > bkey) {
          bkey = kl;
          best = ol;
        }
      }
      lead = best;
      fl = f[ext[best]];
      if (total >= max_visited) {
        nc = total;
        st = kLtsBudget;
        break;
      }
      for (uint32_t q = head, step = 0; q < (uint32_t)n_ext && step < kMaxArrivals;
           q = rec[(size_t)q * kRecWords + 3], step++) {
        if (q == (uint32_t)i) continue;
        const uint32_t *o = rec + (size_t)q * kRecWords;
        const int on = (int)min(o[0], (uint32_t)kLtsMaxVisited);
        for (int j = 0; j < on && nc < kLtsMaxVisited; j++)
          if (o[4 + j] != v) comp[nc++] = o[4 + j];
      }
      bool over = false;
      for (uint32_t q = head, step = 0; q < (uint32_t)n_ext && step < kMaxArrivals && !over;
           q = rec[(size_t)q * kRecWords + 3], step++) {
        if (q == (uint32_t)i) continue;
        const uint32_t *o = rec + (size_t)q * kRecWords;
        const int ow = (int)min(o[1], (uint32_t)kLtsMaxFrontier);
        for (int j = 0; j < ow && !over; j++) {
          const uint32_t u = o[4 + kLtsMaxVisited + j];
          if (u >= g.n || in_comp(u) || waiting(u)) continue;
          wv[nw] = u;
          wk[nw] = key(u);
          over = ++nw > max_frontier;
        }
      }
      for (int k = 0; k < NB && !over; k++) {
        const int64_t u = neighbour<DIM>(g, x, y, z, k);
        if (u < 0 || in_comp((uint32_t)u) || waiting((uint32_t)u)) continue;
        wv[nw] = (uint32_t)u;
        wk[nw] = key(u);
        over = ++nw > max_frontier;
      }
      if (over) {
        st = kLtsBudget;
        break;
      }
      continue;
    }
    if (nc >= max_visited) {
      st = kLtsBudget;
      break;
    }
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] < 0 || nk[k] > kv || waiting((uint32_t)nu[k])) continue;
      wv[nw] = (uint32_t)nu[k];
      wk[nw] = nk[k];
      nw++;
    }
    if (nw > max_frontier) {
      st = kLtsBudget;
      break;
    }
  }
  status[lead] = st;
  saddle[lead] = -1;
  visited[lead] = (uint16_t)nc;
}

uint32_t table_cap(int64_t n_ext) {
  uint32_t cap = 64;
  while ((int64_t)cap < 2 * n_ext) cap <<= 1;
  return cap;
}

}  // namespace

size_t lts_merged_scratch_bytes(int64_t n_ext) {
  return (size_t)n_ext * kRecWords * 4 + (size_t)table_cap(n_ext) * 12;
}

hipError_t launch_lts_merged(const float *f, const uint32_t *rank, int64_t nx, int64_t ny,
                             int64_t nz, const uint32_t *ext, int64_t n_ext, bool maxima,
                             float eps, int max_visited, int max_frontier, uint8_t *status,
                             int32_t *saddle, uint16_t *visited, void *scratch, hipStream_t st) {
  if (n_ext == 0) return hipSuccess;
  if (max_visited < 2 || max_visited > kLtsMaxVisited || max_frontier < 14 ||
      max_frontier > kLtsMaxFrontier || n_ext > kLtsMaxMerged)
    return hipErrorInvalidValue;
  const Grid g{nx, ny, nz, nx * ny * nz};
  const uint32_t cap = table_cap(n_ext);
  uint32_t *rec = (uint32_t *)scratch;
  uint32_t *tkey = rec + (size_t)n_ext * kRecWords, *tcnt = tkey + cap, *thead = tcnt + cap;
  hipLaunchKernelGGL(lts_table_clear_kernel, dim3(std::min<uint32_t>((cap + 255) / 256, 2048)), dim3(256),
                     0, st, tkey, tcnt, thead, cap);
  const dim3 grid((unsigned)((n_ext + 255) / 256)), block(256);
  const uint32_t flip = maxima ? 0u : 0xFFFFFFFFu;
  if (nz > 1)
    hipLaunchKernelGGL(lts_merge_kernel<3>, grid, block, 0, st, f, rank, g, ext, n_ext, flip, eps,
                       max_visited, max_frontier, status, saddle, visited, rec, tkey, tcnt, thead,
                       cap - 1);
  else
    hipLaunchKernelGGL(lts_merge_kernel<2>, grid, block, 0, st, f, rank, g, ext, n_ext, flip, eps,
                       max_visited, max_frontier, status, saddle, visited, rec, tkey, tcnt, thead,
                       cap - 1);
  return hipGetLastError();
}

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
