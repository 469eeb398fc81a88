// Classification and compaction kernels for gfx950 (MI355X).
//
// classify3d: one block = 64 (x) x kTile3Y (y) vertex columns of a level grid,
// marching along z over `zchunk` planes.  Each plane of the tile, plus a halo
// of H samples, is read from HBM once into an LDS ring; every thread keeps the
// 7-point in-plane stencil (centre, +-x, +-y, +(1,1), -(1,1)) of the planes
// z-1, z, z+1 in registers, so a vertex costs 7 LDS reads instead of 15.  The
// 14 neighbour comparisons form the polarity mask, one byte of the
// link-pattern table (staged in LDS) gives the lower/upper link component
// counts, and boundary vertices take a second lookup with their off-grid
// neighbours forced to one side.  Critical flags leave the block as one
// 64-bit ballot word per wave row.
//
// compact: turns the per-level critical bitmask into the ascending list of
// full-resolution indices: a single pass with decoupled look-back over
// chunks whose ids are handed out in start order, then a wave-cooperative
// expansion in which every store instruction writes consecutive entries.
#include "pcrit_internal.h"

namespace pcrit {
namespace {

// Hardware hands consecutive workgroups to the 8 XCDs round-robin; renumber
// them so that each XCD (and its L2) gets a contiguous run of tiles, whose
// halos it then shares.
__device__ __forceinline__ int xcd_block_id() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = b & 7, j = b >> 3;
  return xcd * q + min(xcd, r) + j;
}

__device__ __forceinline__ bool code_is_critical(unsigned code) {
  // regular iff lower == 1, upper == 1 and no hole flag (bit 7); bit 6
  // (boundary) does not matter
  return (code & 0xBFu) != 0x09u;
}

// Boundary vertex with absent-neighbour mask A != 0.  The link in the domain
// is the part of the full neighbour link spanned by the present neighbours.
// Forcing the absent ones to "upper" leaves the lower link as the 0-bits;
// the 1-bits are then the complement of the lower link in the full link
// sphere, whose component count minus one is the lower link's number of
// holes (Alexander duality on the 2-sphere).  Symmetrically for the upper
// link with the absent neighbours forced to "lower".
__device__ __forceinline__ unsigned boundary_code3(const uint8_t *lut,
                                                   unsigned m, unsigned A) {
  const unsigned eL = lut[m | A];
  const unsigned eU = lut[m & ~A & 0x3FFFu];
  const unsigned holes = ((eL >> 3) > 1u) | ((eU & 7u) > 1u);
  return (eL & 7u) | (eU & 0x38u) | 0x40u | (holes << 7);
}

// In 2D the link is a path at the boundary: its parts never have holes.
__device__ __forceinline__ unsigned boundary_code2(const uint8_t *lut,
                                                   unsigned m, unsigned A) {
  return (lut[m | A] & 7u) | (lut[m & ~A & 0x3Fu] & 0x38u) | 0x40u;
}

// Polarity masks.  Bit j is 1 iff neighbour j comes after the centre c in the
// order (value, full-resolution index).  For a neighbour with a larger index
// ("positive" offset: first non-zero of (dz, dy, dx) > 0) that is f >= c,
// for one with a smaller index it is f > c.
__device__ __forceinline__ unsigned mask3(float c, const float *lo,
                                          const float *mid, const float *hi) {
  // lo: (0,0) (-1,0) (0,-1) (-1,-1) of plane z-1
  // mid: (-1,0) (1,0) (0,-1) (0,1) (-1,-1) (1,1) of plane z
  // hi: (0,0) (1,0) (0,1) (1,1) of plane z+1
  unsigned m = 0;
  m |= (unsigned)(lo[0] > c) << 0;
  m |= (unsigned)(lo[1] > c) << 1;
  m |= (unsigned)(lo[2] > c) << 2;
  m |= (unsigned)(lo[3] > c) << 3;
  m |= (unsigned)(mid[0] > c) << 4;
  m |= (unsigned)(mid[1] >= c) << 5;
  m |= (unsigned)(mid[2] > c) << 6;
  m |= (unsigned)(mid[3] >= c) << 7;
  m |= (unsigned)(mid[4] > c) << 8;
  m |= (unsigned)(mid[5] >= c) << 9;
  m |= (unsigned)(hi[0] >= c) << 10;
  m |= (unsigned)(hi[1] >= c) << 11;
  m |= (unsigned)(hi[2] >= c) << 12;
  m |= (unsigned)(hi[3] >= c) << 13;
  return m;
}

__device__ __forceinline__ unsigned mask2(float c, const float *v) {
  // v: (-1,0) (1,0) (0,-1) (0,1) (-1,-1) (1,1)
  unsigned m = 0;
  m |= (unsigned)(v[0] > c) << 0;
  m |= (unsigned)(v[1] >= c) << 1;
  m |= (unsigned)(v[2] > c) << 2;
  m |= (unsigned)(v[3] >= c) << 3;
  m |= (unsigned)(v[4] > c) << 4;
  m |= (unsigned)(v[5] >= c) << 5;
  return m;
}

constexpr unsigned AXM3 = side_mask3(0, -1), AXP3 = side_mask3(0, 1);
constexpr unsigned AYM3 = side_mask3(1, -1), AYP3 = side_mask3(1, 1);
constexpr unsigned AZM3 = side_mask3(2, -1), AZP3 = side_mask3(2, 1);
constexpr unsigned AXM2 = side_mask2(0, -1), AXP2 = side_mask2(0, 1);
constexpr unsigned AYM2 = side_mask2(1, -1), AYP2 = side_mask2(1, 1);

// ---------------------------------------------------------------------------
// 3D classification
// ---------------------------------------------------------------------------
template <int TY, int H, bool PROG>
__global__ __launch_bounds__(64 * TY) void classify3d_kernel(ClassifyArgs a) {
  constexpr int NT = 64 * TY;
  constexpr int TXH = 64 + 2 * H;      // LDS row pitch (floats)
  constexpr int TYH = TY + 2 * H;      // rows per LDS plane
  constexpr int PLANE = TXH * TYH;
  // Planes in the LDS ring.  Step z reads planes z-H .. z+H (the progressive
  // path reaches two planes out) and stores plane z+H+1; the slot it stores
  // into must not be one that a slower wave may still read before the next
  // barrier, including the prologue's reads of planes z0-1 and z0, hence at
  // least 2H+2 slots.
  constexpr int NS = 2 * H + 2;
  constexpr int RPW = (TYH + TY - 1) / TY;  // plane rows loaded per wave
  __shared__ float sp[NS * PLANE];
  __shared__ __attribute__((aligned(16))) uint8_t slut[kLut3Size];
  __shared__ unsigned s_reclass;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int id = xcd_block_id();
  const int tx = id % a.ntx, rest = id / a.ntx;
  const int ty = rest % a.nty, zc = rest / a.nty;
  const int x0 = tx * 64, y0 = ty * TY, z0 = zc * a.zchunk;
  const int z1 = min(z0 + a.zchunk, a.mz);

  // Clear the look-back state of the compaction launched after this kernel.
  for (int i = id * NT + tid; i < a.lb_n; i += (int)gridDim.x * NT)
    a.lb_state[i] = 0ull;
  if (id == 0 && tid == 0) *a.lb_counter = 0u;
  if (PROG && tid == 0) s_reclass = 0u;
  {
    const uint4 *g = reinterpret_cast<const uint4 *>(a.lut);
    uint4 *s = reinterpret_cast<uint4 *>(slut);
    for (int i = tid; i < kLut3Size / 16; i += NT) s[i] = g[i];
  }

  // Plane loader: wave w fetches tile rows w, w+TY, ...; per row the 64
  // lanes read the tile interior (one 256-byte run at stride 1) and lanes
  // 0..2H-1 the halo columns.  Off-grid samples are never read.
  auto load_plane = [&](int z, float (&v)[RPW][2]) {
#pragma unroll
    for (int k = 0; k < RPW; k++) {
      v[k][0] = 0.f;
      v[k][1] = 0.f;
      const int r = w + k * TY;
      const int y = y0 - H + r;
      if (r < TYH && z >= 0 && z < a.mz && y >= 0 && y < a.my) {
        const float *row = a.f + (int64_t)z * a.sz + (int64_t)y * a.sy;
        const int x = x0 + lane;
        if (x < a.mx) v[k][0] = row[(int64_t)x * a.sx];
        if (lane < 2 * H) {
          const int c = lane < H ? lane : 64 + lane;
          const int xh = x0 - H + c;
          if (xh >= 0 && xh < a.mx) v[k][1] = row[(int64_t)xh * a.sx];
        }
      }
    }
  };
  auto store_plane = [&](int slot, const float (&v)[RPW][2]) {
    float *pl = sp + slot * PLANE;
#pragma unroll
    for (int k = 0; k < RPW; k++) {
      const int r = w + k * TY;
      if (r < TYH) {
        pl[r * TXH + H + lane] = v[k][0];
        if (lane < 2 * H) pl[r * TXH + (lane < H ? lane : 64 + lane)] = v[k][1];
      }
    }
  };
  const int cbase = (w + H) * TXH + H + lane;  // this thread's column
  // in-plane stencil: (0,0) (-1,0) (1,0) (0,-1) (0,1) (-1,-1) (1,1)
  auto stencil = [&](int slot, float (&P)[7]) {
    const float *q = sp + slot * PLANE + cbase;
    P[0] = q[0];
    P[1] = q[-1];
    P[2] = q[1];
    P[3] = q[-TXH];
    P[4] = q[TXH];
    P[5] = q[-TXH - 1];
    P[6] = q[TXH + 1];
  };
  auto slot_of = [&](int z) { return (z - z0 + H) % NS; };

  // Prologue: planes z0-H .. z0+H into the ring, two more in flight.
  {
    float pro[2 * H + 1][RPW][2];
#pragma unroll
    for (int i = 0; i < 2 * H + 1; i++) load_plane(z0 - H + i, pro[i]);
#pragma unroll
    for (int i = 0; i < 2 * H + 1; i++) store_plane(i, pro[i]);
  }
  float pfA[RPW][2], pfB[RPW][2];
  load_plane(z0 + H + 1, pfA);
  load_plane(z0 + H + 2, pfB);
  __syncthreads();
  float P0[7], P1[7], P2[7];
  stencil(slot_of(z0 - 1), P0);
  stencil(slot_of(z0), P1);

  const int x = x0 + lane, y = y0 + w;
  const bool col_active = (x < a.mx) && (y < a.my);
  const int64_t col_off = (int64_t)y * a.sy + (int64_t)x * a.sx;
  uint64_t *bits_row = a.bits + (int64_t)y * a.rowwords + (x0 >> 6);
  const int64_t bits_plane = (int64_t)a.my * a.rowwords;

  for (int z = z0; z < z1; z++) {
    stencil(slot_of(z + 1), P2);
    const float c = P1[0];
    const float lo[4] = {P0[0], P0[1], P0[3], P0[5]};
    const float mid[6] = {P1[1], P1[2], P1[3], P1[4], P1[5], P1[6]};
    const float hi[4] = {P2[0], P2[2], P2[4], P2[6]};
    const unsigned m = mask3(c, lo, mid, hi);
    if (col_active && c != c) *a.nan_flag = a.gen;

    // absent neighbours (only waves that touch the level boundary)
    const bool wave_inner = y > 0 && y < a.my - 1 && z > 0 && z < a.mz - 1 &&
                            x0 > 0 && x0 + 64 < a.mx;
    unsigned A = 0;
    if (!wave_inner) {
      A = (x == 0 ? AXM3 : 0u) | (x == a.mx - 1 ? AXP3 : 0u) |
          (y == 0 ? AYM3 : 0u) | (y == a.my - 1 ? AYP3 : 0u) |
          (z == 0 ? AZM3 : 0u) | (z == a.mz - 1 ? AZP3 : 0u);
    }

    bool need = col_active;
    bool old_dirty = false;
    bool crit = false;
    if (PROG) {
      const bool old = col_active && !((x | y | z) & 1);
      if (old) {
        // Level-(k+1) neighbours of an old vertex sit two level-k steps
        // away; its level-(k+1) mask uses them, with the same tie rule.
        const float *qm = sp + slot_of(z - 2) * PLANE + cbase;
        const float *q0 = sp + slot_of(z) * PLANE + cbase;
        const float *qp = sp + slot_of(z + 2) * PLANE + cbase;
        const float flo[4] = {qm[0], qm[-2], qm[-2 * TXH], qm[-2 * TXH - 2]};
        const float fmid[6] = {q0[-2],       q0[2],       q0[-2 * TXH],
                               q0[2 * TXH],  q0[-2 * TXH - 2],
                               q0[2 * TXH + 2]};
        const float fhi[4] = {qp[0], qp[2], qp[2 * TXH], qp[2 * TXH + 2]};
        const unsigned m2 = mask3(c, flo, fmid, fhi);
        // absent at level k+1: beyond the last even coordinate
        const int ex = 2 * ((a.mx - 1) >> 1), ey = 2 * ((a.my - 1) >> 1),
                  ez = 2 * ((a.mz - 1) >> 1);
        const unsigned Afull =
            (x == 0 ? AXM3 : 0u) | (x == a.mx - 1 ? AXP3 : 0u) |
            (y == 0 ? AYM3 : 0u) | (y == a.my - 1 ? AYP3 : 0u) |
            (z == 0 ? AZM3 : 0u) | (z == a.mz - 1 ? AZP3 : 0u);
        const unsigned A2 = (x == 0 ? AXM3 : 0u) | (x == ex ? AXP3 : 0u) |
                            (y == 0 ? AYM3 : 0u) | (y == ey ? AYP3 : 0u) |
                            (z == 0 ? AZM3 : 0u) | (z == ez ? AZP3 : 0u);
        old_dirty = (A2 != Afull) || (((m ^ m2) & ~Afull & 0x3FFFu) != 0u);
        if (!old_dirty) {
          // unchanged: keep the code and the critical status of level k+1
          need = false;
          const int xp = x >> 1, yp = y >> 1, zp = z >> 1;
          const uint64_t wb =
              a.prev_bits[((int64_t)zp * a.prev_my + yp) * a.prev_rowwords +
                          (xp >> 6)];
          crit = (wb >> (xp & 63)) & 1ull;
        }
      }
    }
    if (need) {
      const unsigned code = A == 0u ? (unsigned)slut[m] : boundary_code3(slut, m, A);
      crit = code_is_critical(code);
      a.codes[(int64_t)z * a.sz + col_off] = (uint8_t)code;
    }
    const uint64_t bal = __ballot(crit);
    if (lane == 0 && y < a.my) bits_row[(int64_t)z * bits_plane] = bal;
    if (PROG) {
      const uint64_t d = __ballot(old_dirty);
      if (lane == 0 && d) atomicAdd(&s_reclass, (unsigned)__popcll(d));
    }

    // ring advance: plane z+H+1 into the slot of plane z-H, next loads
    store_plane(slot_of(z + H + 1), pfA);
#pragma unroll
    for (int k = 0; k < RPW; k++) {
      pfA[k][0] = pfB[k][0];
      pfA[k][1] = pfB[k][1];
    }
    load_plane(z + H + 3, pfB);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 7; i++) {
      P0[i] = P1[i];
      P1[i] = P2[i];
    }
  }
  if (PROG) {
    __syncthreads();
    if (tid == 0 && s_reclass) atomicAdd(a.reclass, s_reclass);
  }
}

// ---------------------------------------------------------------------------
// 2D classification: one block = 256 consecutive x of a level row, marching
// along y over `zchunk` rows; 3-row register window of (x-1, x, x+1).
// ---------------------------------------------------------------------------
template <int H, bool PROG>
__global__ __launch_bounds__(kTile2X) void classify2d_kernel(ClassifyArgs a) {
  constexpr int NT = kTile2X;
  constexpr int TXH = kTile2X + 2 * H;
  constexpr int NS = 2 * H + 2;  // LDS ring of rows, sized as in classify3d
  __shared__ float sr[NS * TXH];
  __shared__ uint8_t slut[kLut2Size];
  __shared__ unsigned s_reclass;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int id = xcd_block_id();
  const int tx = id % a.ntx, yc = id / a.ntx;
  const int x0 = tx * kTile2X, y0 = yc * a.zchunk;
  const int y1 = min(y0 + a.zchunk, a.my);

  for (int i = id * NT + tid; i < a.lb_n; i += (int)gridDim.x * NT)
    a.lb_state[i] = 0ull;
  if (id == 0 && tid == 0) *a.lb_counter = 0u;
  if (PROG && tid == 0) s_reclass = 0u;
  if (tid < kLut2Size) slut[tid] = a.lut[tid];

  auto load_row = [&](int y, float (&v)[2]) {
    v[0] = 0.f;
    v[1] = 0.f;
    if (y >= 0 && y < a.my) {
      const float *row = a.f + (int64_t)y * a.sy;
      const int x = x0 + tid;
      if (x < a.mx) v[0] = row[(int64_t)x * a.sx];
      if (tid < 2 * H) {
        const int c = tid < H ? tid : kTile2X + tid;
        const int xh = x0 - H + c;
        if (xh >= 0 && xh < a.mx) v[1] = row[(int64_t)xh * a.sx];
      }
    }
  };
  auto store_row = [&](int slot, const float (&v)[2]) {
    float *r = sr + slot * TXH;
    r[H + tid] = v[0];
    if (tid < 2 * H) r[tid < H ? tid : kTile2X + tid] = v[1];
  };
  auto triple = [&](int slot, float (&R)[3]) {
    const float *q = sr + slot * TXH + H + tid;
    R[0] = q[-1];
    R[1] = q[0];
    R[2] = q[1];
  };
  auto slot_of = [&](int y) { return (y - y0 + H) % NS; };

  {
    float pro[2 * H + 1][2];
#pragma unroll
    for (int i = 0; i < 2 * H + 1; i++) load_row(y0 - H + i, pro[i]);
#pragma unroll
    for (int i = 0; i < 2 * H + 1; i++) store_row(i, pro[i]);
  }
  constexpr int PF = 4;  // rows in flight
  float pf[PF][2];
#pragma unroll
  for (int i = 0; i < PF; i++) load_row(y0 + H + 1 + i, pf[i]);
  __syncthreads();
  float R0[3], R1[3], R2[3];
  triple(slot_of(y0 - 1), R0);
  triple(slot_of(y0), R1);

  const int x = x0 + tid;
  const int xw0 = x0 + 64 * w;
  const bool col_active = x < a.mx;
  const bool wave_x_inner = xw0 > 0 && xw0 + 64 < a.mx;

  for (int y = y0; y < y1; y++) {
    triple(slot_of(y + 1), R2);
    const float c = R1[1];
    const float nb[6] = {R1[0], R1[2], R0[1], R2[1], R0[0], R2[2]};
    const unsigned m = mask2(c, nb);
    if (col_active && c != c) *a.nan_flag = a.gen;
    unsigned A = 0;
    if (!(wave_x_inner && y > 0 && y < a.my - 1)) {
      A = (x == 0 ? AXM2 : 0u) | (x == a.mx - 1 ? AXP2 : 0u) |
          (y == 0 ? AYM2 : 0u) | (y == a.my - 1 ? AYP2 : 0u);
    }
    bool need = col_active, old_dirty = false, crit = false;
    if (PROG) {
      const bool old = col_active && !((x | y) & 1);
      if (old) {
        const float *qm = sr + slot_of(y - 2) * TXH + H + tid;
        const float *q0 = sr + slot_of(y) * TXH + H + tid;
        const float *qp = sr + slot_of(y + 2) * TXH + H + tid;
        const float fn[6] = {q0[-2], q0[2], qm[0], qp[0], qm[-2], qp[2]};
        const unsigned m2 = mask2(c, fn);
        const int ex = 2 * ((a.mx - 1) >> 1), ey = 2 * ((a.my - 1) >> 1);
        const unsigned Afull = (x == 0 ? AXM2 : 0u) |
                               (x == a.mx - 1 ? AXP2 : 0u) |
                               (y == 0 ? AYM2 : 0u) |
                               (y == a.my - 1 ? AYP2 : 0u);
        const unsigned A2 = (x == 0 ? AXM2 : 0u) | (x == ex ? AXP2 : 0u) |
                            (y == 0 ? AYM2 : 0u) | (y == ey ? AYP2 : 0u);
        old_dirty = (A2 != Afull) || (((m ^ m2) & ~Afull & 0x3Fu) != 0u);
        if (!old_dirty) {
          need = false;
          const int xp = x >> 1, yp = y >> 1;
          const uint64_t wb =
              a.prev_bits[(int64_t)yp * a.prev_rowwords + (xp >> 6)];
          crit = (wb >> (xp & 63)) & 1ull;
        }
      }
    }
    if (need) {
      const unsigned code = A == 0u ? (unsigned)slut[m] : boundary_code2(slut, m, A);
      crit = code_is_critical(code);
      a.codes[(int64_t)y * a.sy + (int64_t)x * a.sx] = (uint8_t)code;
    }
    const uint64_t bal = __ballot(crit);
    if (lane == 0 && xw0 < a.mx)
      a.bits[(int64_t)y * a.rowwords + (xw0 >> 6)] = bal;
    if (PROG) {
      const uint64_t d = __ballot(old_dirty);
      if (lane == 0 && d) atomicAdd(&s_reclass, (unsigned)__popcll(d));
    }

    store_row(slot_of(y + H + 1), pf[0]);
#pragma unroll
    for (int i = 0; i + 1 < PF; i++) {
      pf[i][0] = pf[i + 1][0];
      pf[i][1] = pf[i + 1][1];
    }
    load_row(y + H + 1 + PF, pf[PF - 1]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 3; i++) {
      R0[i] = R1[i];
      R1[i] = R2[i];
    }
  }
  if (PROG) {
    __syncthreads();
    if (tid == 0 && s_reclass) atomicAdd(a.reclass, s_reclass);
  }
}

// ---------------------------------------------------------------------------
// Compaction: bitmask -> ascending index list.
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAggregate = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1ull;
constexpr long kSpinLimit = 1L << 26;

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__global__ __launch_bounds__(kCompactThreads) void compact_kernel(CompactArgs a) {
  __shared__ int s_chunk;
  __shared__ int64_t s_wtot[kCompactThreads / 64];
  __shared__ int64_t s_prefix;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_chunk = (int)atomicAdd(a.lb_counter, 1u);
  __syncthreads();
  const int chunk = s_chunk;  // ids follow the order in which blocks start
  const int64_t wfirst = (int64_t)chunk * kChunkWords;
  const int64_t wthr = wfirst + (int64_t)tid * kCompactWordsPerThread;

  uint64_t wd[kCompactWordsPerThread];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < kCompactWordsPerThread; k++) {
    wd[k] = (wthr + k < a.words) ? a.bits[wthr + k] : 0ull;
    cnt += __popcll(wd[k]);
  }
  int incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(incl, d);
    if (lane >= d) incl += v;
  }
  if (lane == 63) s_wtot[w] = incl;
  __syncthreads();
  int64_t woff = 0, btot = 0;
#pragma unroll
  for (int i = 0; i < kCompactThreads / 64; i++) {
    if (i < w) woff += s_wtot[i];
    btot += s_wtot[i];
  }

  if (tid == 0) {
    uint64_t *st = a.lb_state;
    int64_t prefix = 0;
    if (chunk == 0) {
      __hip_atomic_store(&st[0], kFlagPrefix | (uint64_t)btot, __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&st[chunk], kFlagAggregate | (uint64_t)btot,
                         __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      long spins = 0;
      int i = chunk - 1;
      while (i >= 0) {
        const uint64_t v = __hip_atomic_load(&st[i], __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t flag = v >> 62;
        if (flag == 0) {
          // Chunk i belongs to a block that started earlier and waits only
          // on chunks before it, so it publishes in finite time; the limit
          // only guards against a broken invariant.
          if (++spins > kSpinLimit) {
            *a.err_flag = a.gen;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        prefix += (int64_t)(v & kValueMask);
        if (flag == 2) break;
        --i;
      }
      __hip_atomic_store(&st[chunk], kFlagPrefix | (uint64_t)(prefix + btot),
                         __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_prefix = prefix;
  }
  __syncthreads();
  const int64_t base = a.level_base[a.slot];
  const int64_t my_off = base + s_prefix + woff + (incl - cnt);

  if (chunk == a.nchunks - 1 && tid == 0) {
    const int64_t total = s_prefix + btot;
    a.level_base[a.slot + 1] = base + total;
    if (a.count_dev) {
      int64_t out = total;
      if (*a.nan_flag == a.gen) out = -1;
      else if (*a.err_flag == a.gen) out = -2;
      *a.count_dev = out;
    }
  }
  if (chunk == 0 && tid == 0 && a.zero_next) *a.zero_next = 0u;

  // Wave-cooperative expansion of the wave's 256 words, in index order.
  const int64_t gw0 = wfirst + (int64_t)w * 64 * kCompactWordsPerThread;
  if (gw0 >= a.words) return;
  int64_t r = gw0 / a.rowwords;
  int xw = (int)(gw0 - r * a.rowwords);
  int64_t yy = r % a.my, zz = r / a.my;
  const int64_t rowstep = a.s * a.nx;
  int64_t rowbase = rowstep * (yy + a.ny * zz);
  for (int L = 0; L < 64; L++) {
    int64_t off = (int64_t)readlane64((uint64_t)my_off, L);
#pragma unroll
    for (int k = 0; k < kCompactWordsPerThread; k++) {
      const uint64_t word = readlane64(wd[k], L);
      if (word) {
        const unsigned rank = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(word >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)word, 0u));
        if ((word >> lane) & 1ull) {
          const int64_t pos = off + rank;
          if (pos < a.cap) {
            const uint32_t idx =
                (uint32_t)(rowbase + a.s * (int64_t)(xw * 64 + lane));
            a.crit[pos] = idx;
            if (a.crit_codes) a.crit_codes[pos] = a.codes[idx];
          }
        }
        off += __popcll(word);
      }
      if (++xw == a.rowwords) {
        xw = 0;
        if (++yy == a.my) {
          yy = 0;
          ++zz;
        }
        rowbase = rowstep * (yy + a.ny * zz);
      }
    }
    if (gw0 + (int64_t)(L + 1) * kCompactWordsPerThread >= a.words) break;
  }
}

}  // namespace

int classify3d_zchunk(int mx, int my, int mz) {
  const int64_t cols = (int64_t)((mx + 63) / 64) * ((my + kTile3Y - 1) / kTile3Y);
  // aim for >= 16 blocks per CU on 256 CUs, chunks of 16..64 planes
  int zc = 64;
  while (zc > 16 && cols * ((mz + zc - 1) / zc) < 4096) zc >>= 1;
  return zc > mz ? mz : zc;
}

int classify2d_ychunk(int mx, int my) {
  const int64_t cols = (mx + kTile2X - 1) / kTile2X;
  int yc = 256;
  while (yc > 16 && cols * ((my + yc - 1) / yc) < 4096) yc >>= 1;
  return yc > my ? my : yc;
}

hipError_t launch_classify3d(const ClassifyArgs &a, bool progressive,
                             hipStream_t st) {
  const int nzc = (a.mz + a.zchunk - 1) / a.zchunk;
  const dim3 grid((unsigned)(a.ntx * a.nty * nzc));
  if (progressive)
    hipLaunchKernelGGL((classify3d_kernel<kTile3Y, 2, true>), grid,
                       dim3(64 * kTile3Y), 0, st, a);
  else
    hipLaunchKernelGGL((classify3d_kernel<kTile3Y, 1, false>), grid,
                       dim3(64 * kTile3Y), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_classify2d(const ClassifyArgs &a, bool progressive,
                             hipStream_t st) {
  const int nyc = (a.my + a.zchunk - 1) / a.zchunk;
  const dim3 grid((unsigned)(a.ntx * nyc));
  if (progressive)
    hipLaunchKernelGGL((classify2d_kernel<2, true>), grid, dim3(kTile2X), 0,
                       st, a);
  else
    hipLaunchKernelGGL((classify2d_kernel<1, false>), grid, dim3(kTile2X), 0,
                       st, a);
  return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)a.nchunks),
                     dim3(kCompactThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace pcrit
