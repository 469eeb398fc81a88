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
// linear scan behind a 128-bit Bloom filter, which stays cheap for the
// small components that noise extrema have.
//
// lts_propagate_kernel runs every propagation on its own.  The merged
// kernels further down (Section 4.4) let the propagations that meet at a
// saddle go on as one, in rounds.
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

// Grids hold fewer than 2^32 vertices, so indices and coordinates are
// 32-bit (a 64-bit division is a long emulated sequence on the GPU).
struct Grid {
  uint32_t nx, ny, nz, n;
};

__device__ __forceinline__ void coords(const Grid &g, uint32_t v, uint32_t &x, uint32_t &y,
                                       uint32_t &z) {
  const uint32_t q = v / g.nx;
  x = v - q * g.nx;
  z = q / g.ny;
  y = q - z * g.ny;
}

// Neighbour k of vertex (x, y, z), or -1 outside the grid (a coordinate
// below 0 wraps past the grid's extent).
template <int DIM>
__device__ __forceinline__ int64_t neighbour(const Grid &g, uint32_t x, uint32_t y, uint32_t z,
                                             int k) {
  const int8_t *o = DIM == 3 ? kNb3[k] : kNb2[k];
  const uint32_t a = x + o[0], b = y + o[1], c = z + o[2];
  if (a >= g.nx || b >= g.ny || c >= g.nz) return -1;
  return (int64_t)((c * g.ny + b) * g.nx + a);
}

// A 128-bit Bloom filter of the vertices a propagation has taken or let
// wait (a vertex never leaves that set): a clear bit proves a vertex new,
// so the scans of the component and the waiting set run only on a set bit.
__device__ __forceinline__ uint32_t seen_bit(uint32_t u) { return (u * 0x9E3779B1u) >> 25; }
__device__ __forceinline__ void seen_mark(uint64_t &s0, uint64_t &s1, uint32_t u) {
  const uint32_t b = seen_bit(u);
  if (b < 64)
    s0 |= 1ull << b;
  else
    s1 |= 1ull << (b - 64);
}
__device__ __forceinline__ bool seen_maybe(uint64_t s0, uint64_t s1, uint32_t u) {
  const uint32_t b = seen_bit(u);
  return ((b < 64 ? s0 : s1) >> (b & 63)) & 1;
}

// Membership in a[0 .. n): four entries per step, no early exit (the loads
// of a step issue together).  The arrays hold a multiple of four entries,
// so the reads past n stay inside them; their entries are masked out.
constexpr int kWaitCap = kLtsMaxFrontier + 16;  // waiting vertices: up to max_frontier + 14
static_assert(kWaitCap % 4 == 0 && kLtsMaxVisited % 4 == 0, "scans read four entries at a time");
__device__ __forceinline__ bool scan4(const uint32_t *a, int n, uint32_t u) {
  bool f = false;
  for (int j = 0; j < n; j += 4) {
    const uint32_t a0 = a[j], a1 = a[j + 1], a2 = a[j + 2], a3 = a[j + 3];
    f |= (a0 == u) | ((j + 1 < n) & (a1 == u)) | ((j + 2 < n) & (a2 == u)) |
         ((j + 3 < n) & (a3 == u));
  }
  return f;
}

// Index of the largest of k[0 .. n) (n >= 1; the keys are distinct ranks),
// four keys per step, the running maximum in a register.
__device__ __forceinline__ int argmax4(const uint32_t *k, int n) {
  int b = 0;
  uint32_t kb = k[0];
  for (int j = 0; j < n; j += 4) {
    const uint32_t k0 = k[j], k1 = k[j + 1], k2 = k[j + 2], k3 = k[j + 3];
    if (k0 > kb) {
      kb = k0;
      b = j;
    }
    if (j + 1 < n && k1 > kb) {
      kb = k1;
      b = j + 1;
    }
    if (j + 2 < n && k2 > kb) {
      kb = k2;
      b = j + 2;
    }
    if (j + 3 < n && k3 > kb) {
      kb = k3;
      b = j + 3;
    }
  }
  return b;
}

template <int DIM>
__global__ __launch_bounds__(64) void lts_propagate_kernel(
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
  uint32_t wv[kWaitCap], wk[kWaitCap];
  int nc = 1, nw = 0;
  comp[0] = (uint32_t)m;
  uint64_t s0 = 0, s1 = 0;
  seen_mark(s0, s1, (uint32_t)m);
  const float fm = f[m];
  auto key = [&](int64_t u) { return rank[u] ^ flip; };
  auto in_comp = [&](uint32_t u) { return scan4(comp, nc, u); };
  auto waiting = [&](uint32_t u) { return scan4(wv, nw, u); };
  {
    uint32_t x, y, z;
    coords(g, (uint32_t)m, x, y, z);
    for (int k = 0; k < NB; k++) {
      const int64_t u = neighbour<DIM>(g, x, y, z, k);
      if (u < 0) continue;
      wv[nw] = (uint32_t)u;
      wk[nw] = key(u);
      seen_mark(s0, s1, (uint32_t)u);
      nw++;
    }
  }
  uint8_t st = kLtsBudget;
  int32_t sd = -1;
  while (nw > 0) {
    // take the largest waiting vertex
    const int b = argmax4(wk, nw);
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
    uint32_t x, y, z;
    coords(g, (uint32_t)v, x, y, z);
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
      if (!is_saddle && nu[k] >= 0 && nk[k] > kv &&
          !(seen_maybe(s0, s1, (uint32_t)nu[k]) && in_comp((uint32_t)nu[k])))
        is_saddle = true;
    if (is_saddle) {
      st = kLtsSaddle;
      sd = (int32_t)v;
      break;
    }
    if (nc >= max_visited) break;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] < 0 || nk[k] > kv ||
          (seen_maybe(s0, s1, (uint32_t)nu[k]) && waiting((uint32_t)nu[k])))
        continue;
      wv[nw] = (uint32_t)nu[k];
      wk[nw] = nk[k];
      seen_mark(s0, s1, (uint32_t)nu[k]);
      nw++;
    }
    if (nw > max_frontier) break;
  }
  status[i] = st;
  saddle[i] = sd;
  visited[i] = (uint16_t)nc;
}

// Merged propagations (Sections 4.4 and 4.5), in rounds.  Scratch: one
// record per listed extremum (a parked component, its waiting vertices, its
// leader, the next record parked at the same saddle), an open-addressing
// table of saddles (vertex, higher neighbours taken by the arrivals so far,
// the last record parked there), and two queues of completed saddles.
//
// Round 0 runs one propagation per listed extremum up to its first stop.  A
// propagation that stops at a saddle s parks itself, joins s's list and adds
// the higher neighbours of s it holds to s's count; the one whose addition
// completes the count (every higher neighbour of s taken) puts s in the
// queue of the next round, and every propagation of the round ends there.
// Round r + 1 merges every saddle of round r's queue: the union of the
// parked components and waiting sets, led by the largest leader, goes on
// from s until its next stop.  Records, statuses and queue entries of one
// round are read only in a later kernel, so the kernel boundary orders them
// and no fence is needed.  A component merged in round r holds at least
// r + 2 vertices (two parked components share only s, and a propagation
// takes a vertex before it stops again), and a union of max_visited
// vertices stops at the budget, so max_visited rounds after round 0 finish
// every propagation.
constexpr int kRecWords = 4 + kLtsMaxVisited + kLtsMaxFrontier;
static_assert(kRecWords % 4 == 0 && kLtsMaxVisited % 4 == 0, "records of 16-byte blocks");
constexpr uint32_t kNone = 0xFFFFFFFFu;
// arrivals at one saddle: each holds one of its (at most 14) higher neighbours
constexpr uint32_t kMaxArrivals = 16;
constexpr int kRounds = kLtsMaxVisited + 1;  // counters: round 0 .. max_visited

__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  // integer hash "lowbias32" (C. Wellons, hash-prospector)
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return h;
}

struct MergeArgs {
  const float *f;
  const uint32_t *rank;
  Grid g;
  const uint32_t *ext;
  int64_t n_ext;
  uint32_t flip;
  float eps;
  int max_visited, max_frontier;
  uint8_t *status;
  int32_t *saddle;
  uint16_t *visited;
  uint32_t *rec, *tkey, *tcnt, *thead, tmask;
  uint32_t *queue[2];  // round r reads queue[r & 1]
  uint32_t *qcount;    // qcount[r]: entries of round r's queue
};

__global__ __launch_bounds__(256) void lts_table_clear_kernel(uint32_t *tkey, uint32_t *tcnt,
                                                              uint32_t *thead, uint32_t cap,
                                                              uint32_t *qcount) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (uint32_t)kRounds + 1) qcount[t] = 0;
  for (uint32_t j = t; j < cap; j += gridDim.x * blockDim.x) {
    tkey[j] = kNone;
    tcnt[j] = 0;
    thead[j] = kNone;
  }
}

// The per-thread state of one propagation.
struct Prop {
  uint32_t comp[kLtsMaxVisited];
  uint32_t wv[kWaitCap], wk[kWaitCap];
  int nc, nw;
  uint32_t lead;
  float fl;
  uint64_t s0, s1;  // Bloom filter of comp and the waiting vertices
  __device__ void mark(uint32_t u) { seen_mark(s0, s1, u); }
  __device__ bool maybe(uint32_t u) const { return seen_maybe(s0, s1, u); }
  __device__ bool in_comp(uint32_t u) const { return scan4(comp, nc, u); }
  __device__ bool waiting(uint32_t u) const { return scan4(wv, nw, u); }
};

__device__ __forceinline__ void finish(const MergeArgs &a, uint32_t lead, uint8_t st, int nc) {
  a.status[lead] = st;
  a.saddle[lead] = -1;
  a.visited[lead] = (uint16_t)nc;
}

// Run propagation p (record `own`) in round `round` until it stops: the
// leader's final status, or an arrival at a saddle (parked, and the saddle
// queued for the next round when this arrival completes its count).
template <int DIM>
__device__ void advance(const MergeArgs &a, int round, uint32_t own, Prop &p) {
  constexpr int NB = DIM == 3 ? 14 : 6;
  const bool maxima = a.flip == 0u;
  auto key = [&](int64_t u) { return a.rank[u] ^ a.flip; };
  for (;;) {
    if (p.nw == 0) {  // the whole grid taken: nothing ends this extremum
      finish(a, p.lead, kLtsPersistent, p.nc);
      return;
    }
    const int b = argmax4(p.wk, p.nw);
    const uint32_t v = p.wv[b], kv = p.wk[b];
    p.wv[b] = p.wv[p.nw - 1];
    p.wk[b] = p.wk[p.nw - 1];
    p.nw--;
    p.comp[p.nc++] = v;
    const float d = maxima ? p.fl - a.f[v] : a.f[v] - p.fl;
    if (d > a.eps) {
      finish(a, p.lead, kLtsPersistent, p.nc);
      return;
    }
    // taken in decreasing order (a merged component holds the vertices above
    // its saddle, everything waiting lies below), so a smaller neighbour of
    // v is outside the component
    uint32_t x, y, z;
    coords(a.g, (uint32_t)v, x, y, z);
    int64_t nu[NB];
    uint32_t nk[NB];
#pragma unroll
    for (int k = 0; k < NB; k++) {
      nu[k] = neighbour<DIM>(a.g, x, y, z, k);
      nk[k] = nu[k] >= 0 ? key(nu[k]) : 0u;
    }
    uint32_t nh = 0, mine = 0;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] >= 0 && nk[k] > kv) {
        nh++;
        mine += p.maybe((uint32_t)nu[k]) && p.in_comp((uint32_t)nu[k]) ? 1u : 0u;
      }
    }
    if (mine < nh) {  // arrival at the saddle v
      uint32_t *r = a.rec + (size_t)own * kRecWords;
      r[0] = (uint32_t)p.nc;
      r[1] = (uint32_t)p.nw;
      r[2] = p.lead;
      // whole 16-byte blocks: the record is 16-byte aligned (656 bytes), its
      // areas start on block boundaries and hold the last partial block
      // (at most 32 taken, fewer than 128 waiting at an arrival); words past
      // the counts are never read
      for (int j = 0; j < p.nc; j += 4)
        *reinterpret_cast<uint4 *>(r + 4 + j) =
            make_uint4(p.comp[j], p.comp[j + 1], p.comp[j + 2], p.comp[j + 3]);
      for (int j = 0; j < p.nw; j += 4)
        *reinterpret_cast<uint4 *>(r + 4 + kLtsMaxVisited + j) =
            make_uint4(p.wv[j], p.wv[j + 1], p.wv[j + 2], p.wv[j + 3]);
      a.status[p.lead] = kLtsSaddle;  // final unless a merge picks this leader
      a.saddle[p.lead] = (int32_t)v;
      a.visited[p.lead] = (uint16_t)p.nc;
      uint32_t h = mix32(v) & a.tmask;
      for (uint32_t probe = 0; probe <= a.tmask; probe++) {  // at most half full: ends
        const uint32_t k = atomicCAS(&a.tkey[h], kNone, v);
        if (k == kNone || k == v) break;
        h = (h + 1) & a.tmask;
      }
      r[3] = atomicExch(&a.thead[h], own);
      if (atomicAdd(&a.tcnt[h], mine) + mine == nh && round + 1 < kRounds) {
        const uint32_t q = atomicAdd(&a.qcount[round + 1], 1u);
        if (q < (uint32_t)a.n_ext) a.queue[(round + 1) & 1][q] = h;
      }
      return;
    }
    if (p.nc >= a.max_visited) {
      finish(a, p.lead, kLtsBudget, p.nc);
      return;
    }
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (nu[k] < 0 || nk[k] > kv || (p.maybe((uint32_t)nu[k]) && p.waiting((uint32_t)nu[k])))
        continue;
      p.wv[p.nw] = (uint32_t)nu[k];
      p.wk[p.nw] = nk[k];
      p.mark((uint32_t)nu[k]);
      p.nw++;
    }
    if (p.nw > a.max_frontier) {
      finish(a, p.lead, kLtsBudget, p.nc);
      return;
    }
  }
}

// Round 0: one thread per listed extremum.
template <int DIM>
__global__ __launch_bounds__(64) void lts_merge_start_kernel(MergeArgs a) {
  constexpr int NB = DIM == 3 ? 14 : 6;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_ext) return;
  auto key = [&](int64_t u) { return a.rank[u] ^ a.flip; };
  const int64_t m = a.ext[i];
  bool ok = m < a.g.n;
  Prop p;
  p.nc = 1;
  p.nw = 0;
  p.s0 = p.s1 = 0;
  p.mark((uint32_t)m);
  if (ok) {  // the neighbours wait; an extremum of the kind asked for comes after all of them
    uint32_t x, y, z;
    coords(a.g, (uint32_t)m, x, y, z);
    const uint32_t km = key(m);
    for (int k = 0; k < NB; k++) {
      const int64_t u = neighbour<DIM>(a.g, x, y, z, k);
      if (u < 0) continue;
      p.wv[p.nw] = (uint32_t)u;
      p.wk[p.nw] = key(u);
      p.mark((uint32_t)u);
      ok = ok && p.wk[p.nw] < km;
      p.nw++;
    }
  }
  if (!ok) {
    a.status[i] = kLtsInvalid;
    a.saddle[i] = -1;
    a.visited[i] = 0;
    return;
  }
  p.comp[0] = (uint32_t)m;
  p.lead = (uint32_t)i;
  p.fl = a.f[m];
  advance<DIM>(a, 0, (uint32_t)i, p);
}

// Round r >= 1: one thread per saddle completed in round r - 1.
template <int DIM>
__global__ __launch_bounds__(64) void lts_merge_round_kernel(MergeArgs a, int round) {
  constexpr int NB = DIM == 3 ? 14 : 6;
  const uint32_t cnt = min(a.qcount[round], (uint32_t)a.n_ext);
  auto key = [&](int64_t u) { return a.rank[u] ^ a.flip; };
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    const uint32_t h = min(a.queue[round & 1][t], a.tmask);
    const uint32_t v = a.tkey[h], head = a.thead[h];
    if (v >= a.g.n || head >= (uint32_t)a.n_ext) continue;  // never: queued slots hold both
    // every record in the list was parked in an earlier round: index,
    // counts and leader are in range (the clamps only keep a broken
    // invariant from reading past the buffers)
    Prop p;
    int total = 1;
    uint32_t best = kNone, bkey = 0;
    for (uint32_t q = head, step = 0; q < (uint32_t)a.n_ext && step < kMaxArrivals;
         q = a.rec[(size_t)q * kRecWords + 3], step++) {
      const uint32_t *o = a.rec + (size_t)q * kRecWords;
      total += (int)min(o[0], (uint32_t)kLtsMaxVisited) - 1;  // v is in every parked component
      const uint32_t ol = min(o[2], (uint32_t)(a.n_ext - 1));
      const uint32_t kl = key(a.ext[ol]);
      if (best == kNone || kl > bkey) {
        bkey = kl;
        best = ol;
      }
    }
    p.lead = best;
    p.fl = a.f[a.ext[best]];
    if (total >= a.max_visited) {
      finish(a, best, kLtsBudget, total);
      continue;
    }
    p.nc = 0;
    p.nw = 0;
    p.s0 = p.s1 = 0;
    p.comp[p.nc++] = v;
    p.mark(v);
    for (uint32_t q = head, step = 0; q < (uint32_t)a.n_ext && step < kMaxArrivals;
         q = a.rec[(size_t)q * kRecWords + 3], step++) {
      const uint32_t *o = a.rec + (size_t)q * kRecWords;
      const int on = (int)min(o[0], (uint32_t)kLtsMaxVisited);
      for (int j = 0; j < on; j += 4) {  // 16-byte blocks, as written
        const uint4 c4 = *reinterpret_cast<const uint4 *>(o + 4 + j);
        const uint32_t cs[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
        for (int t = 0; t < 4; t++)
          if (j + t < on && cs[t] != v && p.nc < kLtsMaxVisited) {
            p.mark(cs[t]);
            p.comp[p.nc++] = cs[t];
          }
      }
    }
    bool over = false;
    for (uint32_t q = head, step = 0; q < (uint32_t)a.n_ext && step < kMaxArrivals && !over;
         q = a.rec[(size_t)q * kRecWords + 3], step++) {
      const uint32_t *o = a.rec + (size_t)q * kRecWords;
      const int ow = (int)min(o[1], (uint32_t)kLtsMaxFrontier);
      for (int j = 0; j < ow && !over; j += 4) {
        const uint4 f4 = *reinterpret_cast<const uint4 *>(o + 4 + kLtsMaxVisited + j);
        const uint32_t fs[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
        for (int t = 0; t < 4; t++) {
          const uint32_t u = fs[t];
          if (over || j + t >= ow || u >= a.g.n ||
              (p.maybe(u) && (p.in_comp(u) || p.waiting(u))))
            continue;
          p.wv[p.nw] = u;
          p.wk[p.nw] = key(u);
          p.mark(u);
          over = ++p.nw > a.max_frontier;
        }
      }
    }
    uint32_t x, y, z;
    coords(a.g, (uint32_t)v, x, y, z);
    for (int k = 0; k < NB && !over; k++) {  // the saddle's own neighbours
      const int64_t u = neighbour<DIM>(a.g, x, y, z, k);
      if (u < 0 || (p.maybe((uint32_t)u) && (p.in_comp((uint32_t)u) || p.waiting((uint32_t)u))))
        continue;
      p.wv[p.nw] = (uint32_t)u;
      p.wk[p.nw] = key(u);
      p.mark((uint32_t)u);
      over = ++p.nw > a.max_frontier;
    }
    if (over) {
      finish(a, best, kLtsBudget, p.nc);
      continue;
    }
    advance<DIM>(a, round, head, p);  // the merged propagation owns the head record
  }
}

uint32_t table_cap(int64_t n_ext) {
  uint32_t cap = 64;
  while ((int64_t)cap < 2 * n_ext) cap <<= 1;
  return cap;
}

}  // namespace

size_t lts_merged_scratch_bytes(int64_t n_ext) {
  return (size_t)n_ext * kRecWords * 4 + (size_t)table_cap(n_ext) * 12 + (size_t)n_ext * 8 +
         (kRounds + 1) * 4;
}

hipError_t launch_lts_merged(const float *f, const uint32_t *rank, int64_t nx, int64_t ny,
                             int64_t nz, const uint32_t *ext, int64_t n_ext, bool maxima,
                             float eps, int max_visited, int max_frontier, uint8_t *status,
                             int32_t *saddle, uint16_t *visited, void *scratch, hipStream_t st) {
  if (n_ext == 0) return hipSuccess;
  if (max_visited < 2 || max_visited > kLtsMaxVisited || max_frontier < 14 ||
      max_frontier > kLtsMaxFrontier || n_ext > kLtsMaxMerged)
    return hipErrorInvalidValue;
  MergeArgs a;
  a.f = f;
  a.rank = rank;
  a.g = Grid{(uint32_t)nx, (uint32_t)ny, (uint32_t)nz, (uint32_t)(nx * ny * nz)};
  a.ext = ext;
  a.n_ext = n_ext;
  a.flip = maxima ? 0u : 0xFFFFFFFFu;
  a.eps = eps;
  a.max_visited = max_visited;
  a.max_frontier = max_frontier;
  a.status = status;
  a.saddle = saddle;
  a.visited = visited;
  const uint32_t cap = table_cap(n_ext);
  a.rec = (uint32_t *)scratch;
  a.tkey = a.rec + (size_t)n_ext * kRecWords;
  a.tcnt = a.tkey + cap;
  a.thead = a.tcnt + cap;
  a.tmask = cap - 1;
  a.queue[0] = a.thead + cap;
  a.queue[1] = a.queue[0] + n_ext;
  a.qcount = a.queue[1] + n_ext;
  hipLaunchKernelGGL(lts_table_clear_kernel, dim3(std::min<uint32_t>((cap + 255) / 256, 2048)),
                     dim3(256), 0, st, a.tkey, a.tcnt, a.thead, cap, a.qcount);
  // one wave per workgroup: a propagation's wave finishes on its own time
  // (64-lane groups: merged 7.0 -> 6.6 ms against 256-lane groups)
  const dim3 grid((unsigned)((n_ext + 63) / 64)), block(64);
  // rounds: at most 8192 one-wave groups striding over the queue (an empty
  // round is one short launch; a full grid of n_ext threads cost 12 us per
  // empty round)
  const dim3 rgrid((unsigned)std::min<int64_t>(((int64_t)n_ext + 63) / 64, 8192));
  if (nz > 1) {
    hipLaunchKernelGGL(lts_merge_start_kernel<3>, grid, block, 0, st, a);
    for (int r = 1; r <= max_visited; r++)
      hipLaunchKernelGGL(lts_merge_round_kernel<3>, rgrid, block, 0, st, a, r);
  } else {
    hipLaunchKernelGGL(lts_merge_start_kernel<2>, grid, block, 0, st, a);
    for (int r = 1; r <= max_visited; r++)
      hipLaunchKernelGGL(lts_merge_round_kernel<2>, rgrid, block, 0, st, a, r);
  }
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
  const Grid g{(uint32_t)nx, (uint32_t)ny, (uint32_t)nz, (uint32_t)(nx * ny * nz)};
  const dim3 grid((unsigned)((n_ext + 63) / 64)), block(64);
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
