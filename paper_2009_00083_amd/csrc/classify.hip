// Classification and compaction kernels for gfx950 (MI355X).
//
// classify3d / classify2d: per-vertex critical-point classification of one
// level of the hierarchy (wave tiles marched along the slowest axis, see
// below); the result per vertex is a code byte and a bit of the level's
// critical bitmask.
//
// count/expand: turn the per-level critical bitmask into the ascending list
// of full-resolution indices; the expansion is wave-cooperative, so every
// store instruction writes consecutive list entries.
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
// Shared structure of the classification kernels
// ---------------------------------------------------------------------------
// * Every wave owns a tile: 64 consecutive x (one sample per lane) by R rows
//   (3D) or one row (2D), marched along the slowest axis.  The waves of a
//   block share only the link-pattern table, so there is no block barrier
//   inside the march.
// * The samples of a plane stay in registers.  The x-1 and x+1 neighbours
//   come from the lanes next door through DPP wave shifts; lanes 0 and 63
//   take them from a halo load of the same row.
// * A polarity bit is the sign of one float difference, appended to the mask
//   with one alignbit.  For a centre c that is finite and non-zero the sign
//   of c - n (or n - c) is exact, ties included; lanes whose centre is +-0,
//   +-inf or NaN take exact comparisons instead.
// * The march issues global loads only (planes kept three ahead).  On this
//   architecture loads and stores share one completion counter, and with a
//   store in flight the compiler can no longer wait for one particular load;
//   codes and masks are therefore staged in LDS and written after the tile.
// * Persistent blocks walk the tile list; the tiles of one XCD form a
//   contiguous run, so neighbouring tiles (which share halo rows) meet in
//   the same L2.  A launch may cover several small levels (the progressive
//   driver fuses the latency-bound coarse levels); a wave then looks up the
//   level of its tile in the launch's level table.
constexpr int kUnroll = 6;       // march unroll: window period 3, parity 2
constexpr uint8_t kKeep = 0xFF;  // staging: no code to write (never a code)
constexpr int kDppShr1 = 0x138;  // wave_shr:1 -- lane i reads lane i-1
constexpr int kDppShl1 = 0x130;  // wave_shl:1 -- lane i reads lane i+1
constexpr unsigned kPos3 = 0x3EA0u;  // mask bits of positive 3D offsets
constexpr unsigned kPos2 = 0x2Au;    // mask bits of positive 2D offsets

// x-1 neighbour: lane i gets lane i-1, lane 0 gets `halo` (its lane-0 value)
__device__ __forceinline__ float from_left(float halo, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(halo), __float_as_int(v), kDppShr1, 0xF, 0xF, false));
}
// x+1 neighbour: lane i gets lane i+1, lane 63 gets `halo` (its lane-63 value)
__device__ __forceinline__ float from_right(float halo, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(halo), __float_as_int(v), kDppShl1, 0xF, 0xF, false));
}
// m << 1 | sign bit of d
__device__ __forceinline__ unsigned push_sign(unsigned m, float d) {
  return __builtin_amdgcn_alignbit(m, __float_as_uint(d), 31);
}
// +-0, +-inf, NaN: the centres whose differences may not carry the order
__device__ __forceinline__ bool special_centre(float c) {
  return __builtin_amdgcn_classf(c, 0x3 | 0x4 | 0x200 | 0x20 | 0x40);
}

// One plane of a wave tile: rows y0-1 .. y0+R (index i = row - y0 + 1).
template <int R>
struct Plane {
  float v[R + 2];  // samples at x
  float l[R + 2];  // samples at x-1 (rows 0..R used)
  float r[R + 2];  // samples at x+1 (rows 1..R+1 used)
  unsigned pm;     // previous-level masks of the even rows (progressive)
};

template <int R>
struct PlaneLoad {
  float v[R + 2];
  float h[R + 2];  // lane 0: x0-1, lane 63: x0+64, other lanes: x again
  unsigned pm[(R + 1) / 2];
};

// Level-(k+1) polarity mask of an old vertex, from its neighbours two
// level-k steps away (used where the previous level's masks are not
// stored); same tie rule as the level-k mask.  Off-grid positions are
// clamped: their bits are masked by the caller.
__device__ __forceinline__ unsigned far_mask3(const float *f,
                                              const LevelDesc &g, int x,
                                              int y, int z, float c) {
  float v[14];
#pragma unroll
  for (int j = 0; j < 14; j++) {
    const int xx = min(max(x + 2 * kOff3[j][0], 0), g.mx - 1);
    const int yy = min(max(y + 2 * kOff3[j][1], 0), g.my - 1);
    const int zz = min(max(z + 2 * kOff3[j][2], 0), g.mz - 1);
    v[j] = f[(int64_t)xx * g.sx + (int64_t)yy * g.sy + (int64_t)zz * g.sz];
  }
  const float lo[4] = {v[0], v[1], v[2], v[3]};
  const float mid[6] = {v[4], v[5], v[6], v[7], v[8], v[9]};
  const float hi[4] = {v[10], v[11], v[12], v[13]};
  return mask3(c, lo, mid, hi);
}

__device__ __forceinline__ unsigned far_mask2(const float *f,
                                              const LevelDesc &g, int x,
                                              int y, float c) {
  float v[6];
#pragma unroll
  for (int j = 0; j < 6; j++) {
    const int xx = min(max(x + 2 * kOff2[j][0], 0), g.mx - 1);
    const int yy = min(max(y + 2 * kOff2[j][1], 0), g.my - 1);
    v[j] = f[(int64_t)xx * g.sx + (int64_t)yy * g.sy];
  }
  return mask2(c, v);
}

// Absent-neighbour mask of (x, y, z) on a level of size (mx, my, mz), and
// the same on the next coarser level for an old vertex (its neighbours two
// steps away: absent beyond the last even coordinate).
__device__ __forceinline__ unsigned absent3(int x, int y, int z, int mx,
                                            int my, int mz) {
  return (x == 0 ? AXM3 : 0u) | (x == mx - 1 ? AXP3 : 0u) |
         (y == 0 ? AYM3 : 0u) | (y == my - 1 ? AYP3 : 0u) |
         (z == 0 ? AZM3 : 0u) | (z == mz - 1 ? AZP3 : 0u);
}
__device__ __forceinline__ unsigned absent2(int x, int y, int mx, int my) {
  return (x == 0 ? AXM2 : 0u) | (x == mx - 1 ? AXP2 : 0u) |
         (y == 0 ? AYM2 : 0u) | (y == my - 1 ? AYP2 : 0u);
}

// ---------------------------------------------------------------------------
// 3D: one wave tile (64 x R x zchunk) of level g.
//   RP:  the previous level's masks are stored (g.prev_masks)
//   WM:  the level's masks may be stored for the next level (g.masks)
//   FAR: the previous level's masks may be computed from the field
// stc / stm: this wave's LDS staging for codes / masks.
// ---------------------------------------------------------------------------
template <int R, bool RP, bool WM, bool FAR>
__device__ __forceinline__ void tile3d(const ClassifyArgs &a,
                                       const LevelDesc &g, int t, int lane,
                                       const uint8_t *slut, uint8_t *stc,
                                       uint16_t *stm, bool &nan_seen,
                                       unsigned &reclass) {
  constexpr int NR = R + 2;
  constexpr int U = kUnroll;
  const int tx = t % g.ntx, rest = t / g.ntx;
  const int ty = rest % g.nty, zc = rest / g.nty;
  const int x0 = tx * 64, y0 = ty * R, z0 = zc * g.zchunk;
  const int z1 = min(z0 + g.zchunk, g.mz);
  const int x = x0 + lane;
  const bool col = x < g.mx;
  const bool dirty_test = (RP || FAR) && g.dirty;
  const bool store_masks = WM && g.masks != nullptr;

  // Clamped, unconditional loads (a clamped sample is never used: the
  // absent-neighbour mask covers every off-grid position).
  const int xc = min(x, g.mx - 1);
  const int xh = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + 64, g.mx - 1) : xc);
  const int64_t xoff = (int64_t)xc * g.sx, hoff = (int64_t)xh * g.sx;
  int64_t yoff[NR];
#pragma unroll
  for (int i = 0; i < NR; i++)
    yoff[i] = (int64_t)min(max(y0 - 1 + i, 0), g.my - 1) * g.sy;
  const int pxc = RP ? min(xc >> 1, g.pmx - 1) : 0;
  const uint16_t *pmasks = reinterpret_cast<const uint16_t *>(g.prev_masks);

  auto load = [&](int z, PlaneLoad<R> &d) {
    const int zcl = min(max(z, 0), g.mz - 1);
    const float *pl = a.f + (int64_t)zcl * g.sz;
#pragma unroll
    for (int i = 0; i < NR; i++) {
      d.v[i] = pl[yoff[i] + xoff];
      d.h[i] = pl[yoff[i] + hoff];
    }
    if (RP) {
      const int pz = zcl >> 1;
#pragma unroll
      for (int k = 0; k < (R + 1) / 2; k++) {
        const int py = min((y0 + 2 * k) >> 1, g.pmy - 1);
        d.pm[k] = pmasks[((int64_t)pz * g.pmy + py) * g.pmx + pxc];
      }
    }
  };
  auto derive = [&](const PlaneLoad<R> &d, Plane<R> &p) {
#pragma unroll
    for (int i = 0; i < NR; i++) p.v[i] = d.v[i];
#pragma unroll
    for (int i = 0; i <= R; i++) p.l[i] = from_left(d.h[i], d.v[i]);
#pragma unroll
    for (int i = 1; i <= R + 1; i++) p.r[i] = from_right(d.h[i], d.v[i]);
    if (RP) {
      unsigned pm = 0;
#pragma unroll
      for (int k = 0; k < (R + 1) / 2; k++) pm |= d.pm[k] << (16 * k);
      p.pm = pm;
    }
  };

  uint64_t wbits = 0;  // lane q holds the critical word of staged row q

  // Classify the R vertices of plane z in this lane's column.
  auto step = [&](int z, const Plane<R> &lo, const Plane<R> &mid,
                  const Plane<R> &hi) {
    const bool zlive = z < z1;
#pragma unroll
    for (int j = 0; j < R; j++) {
      const int i = j + 1;
      const int y = y0 + j;
      const bool live = zlive && col && y < g.my;
      const float c = mid.v[i];
      unsigned m = 0;
      m = push_sign(m, hi.r[i + 1] - c);   // 13 (1,1,1)
      m = push_sign(m, hi.v[i + 1] - c);   // 12 (0,1,1)
      m = push_sign(m, hi.r[i] - c);       // 11 (1,0,1)
      m = push_sign(m, hi.v[i] - c);       // 10 (0,0,1)
      m = push_sign(m, mid.r[i + 1] - c);  //  9 (1,1,0)
      m = push_sign(m, c - mid.l[i - 1]);  //  8 (-1,-1,0)
      m = push_sign(m, mid.v[i + 1] - c);  //  7 (0,1,0)
      m = push_sign(m, c - mid.v[i - 1]);  //  6 (0,-1,0)
      m = push_sign(m, mid.r[i] - c);      //  5 (1,0,0)
      m = push_sign(m, c - mid.l[i]);      //  4 (-1,0,0)
      m = push_sign(m, c - lo.l[i - 1]);   //  3 (-1,-1,-1)
      m = push_sign(m, c - lo.v[i - 1]);   //  2 (0,-1,-1)
      m = push_sign(m, c - lo.l[i]);       //  1 (-1,0,-1)
      m = push_sign(m, c - lo.v[i]);       //  0 (0,0,-1)
      m ^= kPos3;
      if (special_centre(c)) {
        const float lov[4] = {lo.v[i], lo.l[i], lo.v[i - 1], lo.l[i - 1]};
        const float midv[6] = {mid.l[i],     mid.r[i],     mid.v[i - 1],
                               mid.v[i + 1], mid.l[i - 1], mid.r[i + 1]};
        const float hiv[4] = {hi.v[i], hi.r[i], hi.v[i + 1], hi.r[i + 1]};
        m = mask3(c, lov, midv, hiv);
        nan_seen |= live && (c != c);
      }
      // absent neighbours, only in waves that touch the level boundary
      const bool inner = y > 0 && y < g.my - 1 && z > 0 && z < g.mz - 1 &&
                         x0 > 0 && x0 + 64 < g.mx;
      const unsigned A = inner ? 0u : absent3(x, y, z, g.mx, g.my, g.mz);
      const unsigned code = A == 0u ? (unsigned)slut[m] : boundary_code3(slut, m, A);
      uint8_t out = live ? (uint8_t)code : kKeep;
      if ((RP || FAR) && dirty_test && !(j & 1) && !(z & 1)) {
        // old vertex (present at level k+1): re-classified only if its
        // polarity mask or its set of absent neighbours changed
        const bool old = live && !(x & 1);
        const unsigned Af = absent3(x, y, z, g.mx, g.my, g.mz);
        const unsigned A2 =
            absent3(x, y, z, 2 * ((g.mx - 1) >> 1) + 1,
                    2 * ((g.my - 1) >> 1) + 1, 2 * ((g.mz - 1) >> 1) + 1);
        unsigned pm = 0;
        if (RP) pm = (mid.pm >> (16 * (j >> 1))) & 0xFFFFu;
        if (FAR && !RP && old) pm = far_mask3(a.f, g, x, y, z, c);
        const bool dirty =
            old && (A2 != Af || ((m ^ pm) & ~Af & 0x3FFFu) != 0u);
        if (old && !dirty && g.keep_clean) out = kKeep;
        reclass += (unsigned)__popcll(__ballot(dirty));
      }
      const int q = (z - z0) * R + j;
      stc[q * 64 + lane] = out;
      if (WM && store_masks) stm[q * 64 + lane] = (uint16_t)m;
      const uint64_t bal = __ballot(live && code_is_critical(code));
      wbits = lane == q ? bal : wbits;
    }
  };

  // Prologue: planes z0-1, z0 derived; z0+1 .. z0+3 in flight.
  Plane<R> W[3];
  PlaneLoad<R> pf[3];
  {
    PlaneLoad<R> d0, d1;
    load(z0 - 1, d0);
    load(z0, d1);
#pragma unroll
    for (int s = 0; s < 3; s++) load(z0 + 1 + s, pf[s]);
    derive(d0, W[0]);
    derive(d1, W[1]);
  }
  // zchunk is a multiple of U; a short last tile runs up to U-1 extra steps
  // whose staged rows are never written out.
  for (int zb = z0; zb < z1; zb += U) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int z = zb + u;
      derive(pf[u % 3], W[(u + 2) % 3]);  // plane z+1
      load(z + 4, pf[u % 3]);
      step(z, W[u % 3], W[(u + 1) % 3], W[(u + 2) % 3]);
    }
  }

  // Write the staged tile.  Rows of a full-width tile at stride 1 leave as
  // dwords (16 lanes per 64-byte row); rows that may hold a kept code,
  // partial tiles and strided levels byte by byte.
  const int nrows = (z1 - z0) * R;
  if (g.write_codes) {
    const bool wide = g.sx == 1 && x0 + 64 <= g.mx && (g.sy & 3) == 0 &&
                      ((uintptr_t)a.codes & 3) == 0;
    auto row_needs_bytes = [&](int q) {
      const int z = z0 + q / R, j = q % R;
      return !wide || (g.keep_clean && !(z & 1) && !(j & 1));
    };
    for (int qb = 0; qb < nrows; qb += 4) {
      const int q = qb + (lane >> 4), part = lane & 15;
      const int y = y0 + q % R, z = z0 + q / R;
      if (q < nrows && y < g.my && !row_needs_bytes(q)) {
        const uint32_t v4 = *reinterpret_cast<const uint32_t *>(stc + q * 64 + part * 4);
        *reinterpret_cast<uint32_t *>(a.codes + (int64_t)z * g.sz +
                                      (int64_t)y * g.sy + x0 + part * 4) = v4;
      }
    }
    for (int q = 0; q < nrows; q++) {
      const int y = y0 + q % R, z = z0 + q / R;
      if (y < g.my && row_needs_bytes(q)) {
        const uint8_t b = stc[q * 64 + lane];
        if (b != kKeep)
          a.codes[(int64_t)z * g.sz + (int64_t)y * g.sy + (int64_t)x * g.sx] = b;
      }
    }
  }
  if (g.lcodes) {
    for (int q = 0; q < nrows; q++) {
      const int y = y0 + q % R, z = z0 + q / R;
      if (y < g.my && col)
        g.lcodes[((int64_t)z * g.my + y) * g.mx + x] = stc[q * 64 + lane];
    }
  }
  {
    const int y = y0 + lane % R, z = z0 + lane / R;
    if (lane < nrows && y < g.my)
      g.bits[((int64_t)z * g.my + y) * g.rowwords + tx] = wbits;
  }
  if (WM && store_masks) {
    uint16_t *om = reinterpret_cast<uint16_t *>(g.masks);
    for (int q = 0; q < nrows; q++) {
      const int y = y0 + q % R, z = z0 + q / R;
      if (y < g.my && col) om[((int64_t)z * g.my + y) * g.mx + x] = stm[q * 64 + lane];
    }
  }
}

// ---------------------------------------------------------------------------
// 2D: one wave tile (64 x zchunk rows) of level g, marched along y.
// ---------------------------------------------------------------------------
struct Row2 {
  float v, l, r;
  unsigned pm;
};
struct RowLoad2 {
  float v, h;
  unsigned pm;
};

template <bool RP, bool WM, bool FAR>
__device__ __forceinline__ void tile2d(const ClassifyArgs &a,
                                       const LevelDesc &g, int t, int lane,
                                       const uint8_t *slut, uint8_t *stc,
                                       uint8_t *stm, bool &nan_seen,
                                       unsigned &reclass) {
  constexpr int U = kUnroll;
  constexpr int PF = 6;  // rows in flight
  const int tx = t % g.ntx, yc = t / g.ntx;
  const int x0 = tx * 64, y0 = yc * g.zchunk;
  const int y1 = min(y0 + g.zchunk, g.my);
  const int x = x0 + lane;
  const bool col = x < g.mx;
  const bool dirty_test = (RP || FAR) && g.dirty;
  const bool store_masks = WM && g.masks != nullptr;
  const int xc = min(x, g.mx - 1);
  const int xh = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + 64, g.mx - 1) : xc);
  const int64_t xoff = (int64_t)xc * g.sx, hoff = (int64_t)xh * g.sx;
  const int pxc = RP ? min(xc >> 1, g.pmx - 1) : 0;
  const uint8_t *pmasks = reinterpret_cast<const uint8_t *>(g.prev_masks);

  auto load = [&](int y, RowLoad2 &d) {
    const int ycl = min(max(y, 0), g.my - 1);
    const float *row = a.f + (int64_t)ycl * g.sy;
    d.v = row[xoff];
    d.h = row[hoff];
    if (RP) d.pm = pmasks[(int64_t)min(ycl >> 1, g.pmy - 1) * g.pmx + pxc];
  };
  auto derive = [&](const RowLoad2 &d, Row2 &p) {
    p.v = d.v;
    p.l = from_left(d.h, d.v);
    p.r = from_right(d.h, d.v);
    if (RP) p.pm = d.pm;
  };
  uint64_t wbits = 0;

  auto step = [&](int y, const Row2 &lo, const Row2 &mid, const Row2 &hi) {
    const bool live = y < y1 && col;
    const float c = mid.v;
    unsigned m = 0;
    m = push_sign(m, hi.r - c);   // 5 (1,1)
    m = push_sign(m, c - lo.l);   // 4 (-1,-1)
    m = push_sign(m, hi.v - c);   // 3 (0,1)
    m = push_sign(m, c - lo.v);   // 2 (0,-1)
    m = push_sign(m, mid.r - c);  // 1 (1,0)
    m = push_sign(m, c - mid.l);  // 0 (-1,0)
    m ^= kPos2;
    if (special_centre(c)) {
      const float nb[6] = {mid.l, mid.r, lo.v, hi.v, lo.l, hi.r};
      m = mask2(c, nb);
      nan_seen |= live && (c != c);
    }
    const bool inner = y > 0 && y < g.my - 1 && x0 > 0 && x0 + 64 < g.mx;
    const unsigned A = inner ? 0u : absent2(x, y, g.mx, g.my);
    const unsigned code = A == 0u ? (unsigned)slut[m] : boundary_code2(slut, m, A);
    uint8_t out = live ? (uint8_t)code : kKeep;
    if ((RP || FAR) && dirty_test && !(y & 1)) {
      const bool old = live && !(x & 1);
      const unsigned Af = absent2(x, y, g.mx, g.my);
      const unsigned A2 = absent2(x, y, 2 * ((g.mx - 1) >> 1) + 1,
                                  2 * ((g.my - 1) >> 1) + 1);
      unsigned pm = 0;
      if (RP) pm = mid.pm;
      if (FAR && !RP && old) pm = far_mask2(a.f, g, x, y, c);
      const bool dirty = old && (A2 != Af || ((m ^ pm) & ~Af & 0x3Fu) != 0u);
      if (old && !dirty && g.keep_clean) out = kKeep;
      reclass += (unsigned)__popcll(__ballot(dirty));
    }
    const int q = y - y0;
    stc[q * 64 + lane] = out;
    if (WM && store_masks) stm[q * 64 + lane] = (uint8_t)m;
    const uint64_t bal = __ballot(live && code_is_critical(code));
    wbits = lane == q ? bal : wbits;
  };

  Row2 W[3];
  RowLoad2 pf[PF];
  {
    RowLoad2 d0, d1;
    load(y0 - 1, d0);
    load(y0, d1);
#pragma unroll
    for (int s = 0; s < PF; s++) load(y0 + 1 + s, pf[s]);
    derive(d0, W[0]);
    derive(d1, W[1]);
  }
  for (int yb = y0; yb < y1; yb += U) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int y = yb + u;
      derive(pf[u % PF], W[(u + 2) % 3]);
      load(y + 1 + PF, pf[u % PF]);
      step(y, W[u % 3], W[(u + 1) % 3], W[(u + 2) % 3]);
    }
  }

  const int nrows = y1 - y0;
  if (g.write_codes) {
    const bool wide = g.sx == 1 && x0 + 64 <= g.mx && (g.sy & 3) == 0 &&
                      ((uintptr_t)a.codes & 3) == 0;
    for (int qb = 0; qb < nrows; qb += 4) {
      const int q = qb + (lane >> 4), part = lane & 15;
      const int y = y0 + q;
      if (q < nrows && wide && !(g.keep_clean && !(y & 1))) {
        const uint32_t v4 = *reinterpret_cast<const uint32_t *>(stc + q * 64 + part * 4);
        *reinterpret_cast<uint32_t *>(a.codes + (int64_t)y * g.sy + x0 + part * 4) = v4;
      }
    }
    for (int q = 0; q < nrows; q++) {
      const int y = y0 + q;
      if (!wide || (g.keep_clean && !(y & 1))) {
        const uint8_t b = stc[q * 64 + lane];
        if (b != kKeep) a.codes[(int64_t)y * g.sy + (int64_t)x * g.sx] = b;
      }
    }
  }
  if (g.lcodes) {
    for (int q = 0; q < nrows; q++)
      if (col) g.lcodes[(int64_t)(y0 + q) * g.mx + x] = stc[q * 64 + lane];
  }
  if (lane < nrows) g.bits[(int64_t)(y0 + lane) * g.rowwords + tx] = wbits;
  if (WM && store_masks) {
    uint8_t *om = reinterpret_cast<uint8_t *>(g.masks);
    for (int q = 0; q < nrows; q++)
      if (col) om[(int64_t)(y0 + q) * g.mx + x] = stm[q * 64 + lane];
  }
}

// ---------------------------------------------------------------------------
// Classification kernels.  A block = kWavesPerBlock independent waves that
// share the link-pattern table in LDS; each wave walks wave tiles of the
// launch's levels (one level, or the fused small levels).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int level_of_tile(const ClassifyArgs &a, int t) {
  int l = 0;
  while (l + 1 < a.nl && t >= a.lv[l + 1].tile_begin) l++;
  return l;
}

template <bool RP, bool WM, bool FAR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void classify3d_kernel(
    ClassifyArgs a) {
  constexpr int NW = kWavesPerBlock;
  constexpr int R = kTile3Y;
  constexpr int ZC = kZChunk3;
  static_assert(ZC % kUnroll == 0, "tile depth must be a multiple of the unroll");
  static_assert(ZC * R <= 64, "one critical word per lane");
  static_assert(R % 2 == 0, "tiles start on even rows");
  __shared__ __attribute__((aligned(16))) uint8_t slut[kLut3Size];
  __shared__ __attribute__((aligned(16))) uint8_t scode[NW][ZC * R * 64];
  __shared__ __attribute__((aligned(16))) uint16_t smask[WM ? NW : 1][WM ? ZC * R * 64 : 2];
  __shared__ unsigned s_reclass[kMaxFused];

  // the wave index is the same in every lane: keep tile arithmetic scalar
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  {
    const uint4 *g = reinterpret_cast<const uint4 *>(a.lut);
    uint4 *s = reinterpret_cast<uint4 *>(slut);
    for (int i = tid; i < kLut3Size / 16; i += 64 * NW) s[i] = g[i];
  }
  if (tid < kMaxFused) s_reclass[tid] = 0u;
  __syncthreads();

  bool nan_seen = false;
  const int nwaves = (int)gridDim.x * NW;
  for (int t = xcd_block_id() * NW + w; t < a.ntiles; t += nwaves) {
    const int l = a.nl == 1 ? 0 : level_of_tile(a, t);
    unsigned reclass = 0;  // wave-uniform
    tile3d<R, RP, WM, FAR>(a, a.lv[l], t - a.lv[l].tile_begin, lane, slut,
                           scode[w], smask[WM ? w : 0], nan_seen, reclass);
    if ((RP || FAR) && lane == 0 && reclass) atomicAdd(&s_reclass[l], reclass);
  }
  if (__ballot(nan_seen) && lane == 0) *a.nan_flag = a.gen;
  __syncthreads();
  if ((RP || FAR) && tid < a.nl)
    a.reclass_part[(int64_t)blockIdx.x * kMaxFused + tid] = s_reclass[tid];
}

template <bool RP, bool WM, bool FAR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void classify2d_kernel(
    ClassifyArgs a) {
  constexpr int NW = kWavesPerBlock;
  constexpr int YC = kYChunk2;
  static_assert(YC % kUnroll == 0 && YC <= 64, "tile depth");
  __shared__ uint8_t slut[kLut2Size];
  __shared__ __attribute__((aligned(16))) uint8_t scode[NW][YC * 64];
  __shared__ uint8_t smask[WM ? NW : 1][WM ? YC * 64 : 4];
  __shared__ unsigned s_reclass[kMaxFused];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < kLut2Size) slut[tid] = a.lut[tid];
  if (tid < kMaxFused) s_reclass[tid] = 0u;
  __syncthreads();

  bool nan_seen = false;
  const int nwaves = (int)gridDim.x * NW;
  for (int t = xcd_block_id() * NW + w; t < a.ntiles; t += nwaves) {
    const int l = a.nl == 1 ? 0 : level_of_tile(a, t);
    unsigned reclass = 0;
    tile2d<RP, WM, FAR>(a, a.lv[l], t - a.lv[l].tile_begin, lane, slut,
                        scode[w], smask[WM ? w : 0], nan_seen, reclass);
    if ((RP || FAR) && lane == 0 && reclass) atomicAdd(&s_reclass[l], reclass);
  }
  if (__ballot(nan_seen) && lane == 0) *a.nan_flag = a.gen;
  __syncthreads();
  if ((RP || FAR) && tid < a.nl)
    a.reclass_part[(int64_t)blockIdx.x * kMaxFused + tid] = s_reclass[tid];
}

// ---------------------------------------------------------------------------
// Compaction: bitmask -> ascending index list, in two passes without atomics
// or waiting: count_kernel stores the number of set bits of every chunk of
// WPT * 256 words; expand_kernel sums the counts of the chunks before its
// own, then writes the indices of its chunk.  Chunks are numbered in list
// order (levels coarse to fine, then index order), so one sum places every
// level's list after the coarser ones.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *scratch) {
  // scratch: kCompactThreads / 64 entries
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < kCompactThreads / 64; i++) s += scratch[i];
  __syncthreads();
  return s;
}

__device__ __forceinline__ int level_of_chunk(const CompactArgs &a, int c) {
  int l = 0;
  while (l + 1 < a.nl && c >= a.lv[l + 1].chunk_begin) l++;
  return l;
}

template <int WPT>
__global__ __launch_bounds__(kCompactThreads) void count_kernel(CompactArgs a) {
  __shared__ int s_red[kCompactThreads / 64];
  const int chunk = blockIdx.x, tid = threadIdx.x;
  const CompactLevel &L = a.lv[level_of_chunk(a, chunk)];
  const int64_t wthr = (int64_t)(chunk - L.chunk_begin) * (kCompactThreads * WPT) +
                       (int64_t)tid * WPT;
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < WPT; k++)
    if (wthr + k < L.words) cnt += __popcll(L.bits[wthr + k]);
  const int tot = block_sum(cnt, s_red);
  if (tid == 0) a.counts[chunk] = tot;
}

template <int WPT>
__global__ __launch_bounds__(kCompactThreads) void expand_kernel(CompactArgs a) {
  constexpr int CW = kCompactThreads * WPT;
  __shared__ int64_t s_red[kCompactThreads / 64];
  __shared__ unsigned s_ured[kCompactThreads / 64];
  __shared__ int s_wtot[kCompactThreads / 64];
  const int chunk = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = level_of_chunk(a, chunk);
  const CompactLevel &L = a.lv[li];
  const int lchunk = chunk - L.chunk_begin;
  // entries before this chunk, and before this chunk's level, in this launch
  int64_t part = 0, lpart = 0;
  for (int i = tid; i < chunk; i += kCompactThreads) {
    const int n = a.counts[i];
    part += n;
    lpart += i < L.chunk_begin ? n : 0;
  }
  const int64_t prefix = block_sum(part, s_red);
  const int64_t lprefix = block_sum(lpart, s_red);
  // lists of earlier launches end at level_base[first slot of this launch]
  const int64_t base = a.level_base[a.lv[0].slot];
  if (lchunk == 0 && L.reclass_out) {
    unsigned r = 0;
    for (int i = tid; i < a.reclass_blocks; i += kCompactThreads)
      r += a.reclass_part[(int64_t)i * kMaxFused + li];
    r = block_sum(r, s_ured);
    if (tid == 0) *L.reclass_out = r;
  }

  const int64_t wfirst = (int64_t)lchunk * CW;
  const int64_t wthr = wfirst + (int64_t)tid * WPT;
  uint64_t wd[WPT];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < WPT; k++) {
    wd[k] = (wthr + k < L.words) ? L.bits[wthr + k] : 0ull;
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
  const int64_t my_off = base + prefix + woff + (incl - cnt);

  // the first chunk of a later level opens its list, the last chunk of the
  // launch closes the last one
  if (li > 0 && lchunk == 0 && tid == 0) a.level_base[L.slot] = base + prefix;
  if (chunk == a.nchunks - 1 && tid == 0) {
    const int64_t total = prefix + btot;
    a.level_base[L.slot + 1] = base + total;
    if (a.count_dev)
      *a.count_dev = (*a.nan_flag == a.gen) ? -1 : total - lprefix;
  }

  // Wave-cooperative expansion of the wave's words, in index order: a word
  // becomes the execution mask (its set lanes are the critical x), and its
  // lanes write consecutive list entries with one store.
  const int64_t gw0 = wfirst + (int64_t)w * 64 * WPT;
  if (gw0 >= L.words) return;
  int64_t r = gw0 / L.rowwords;
  int xw = (int)(gw0 - r * L.rowwords);
  int64_t yy = r % L.my, zz = r / L.my;
  const int64_t rowstep = L.s * a.nx;
  int64_t rowbase = rowstep * (yy + a.ny * zz);
  const uint32_t lane_x = (uint32_t)(L.s * lane);
  const int nw = (int)min((int64_t)64 * WPT, L.words - gw0);
  for (int i = 0; i * WPT < nw; i++) {
    int64_t off = (int64_t)readlane64((uint64_t)my_off, i);
#pragma unroll
    for (int k = 0; k < WPT; k++) {
      const uint64_t word = readlane64(wd[k], i);
      if (word) {
        if (__builtin_amdgcn_inverse_ballot_w64(word)) {
          const unsigned rank = __builtin_amdgcn_mbcnt_hi(
              (unsigned)(word >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)word, 0u));
          const int64_t pos = off + rank;
          if (pos < a.cap) {
            const uint32_t idx = (uint32_t)(rowbase + L.s * (int64_t)xw * 64) + lane_x;
            a.crit[pos] = idx;
            if (a.crit_codes) {
              if (L.lcodes)
                a.crit_codes[pos] =
                    L.lcodes[(yy + (int64_t)L.my * zz) * L.mx + xw * 64 + lane];
              else
                a.crit_codes[pos] = a.codes[idx];
            }
          }
        }
        off += __popcll(word);
      }
      if (++xw == L.rowwords) {
        xw = 0;
        if (++yy == L.my) {
          yy = 0;
          ++zz;
        }
        rowbase = rowstep * (yy + a.ny * zz);
      }
    }
  }
}

// Persistent grid size: resident blocks per CU x CUs, at most 8 per CU.
template <typename K>
int persistent_blocks(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) !=
          hipSuccess)
    return 256;
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  return cus * per_cu;
}

template <typename K>
hipError_t launch_persistent(K kernel, const ClassifyArgs &a, hipStream_t st,
                             int *grid_out) {
  const int threads = 64 * kWavesPerBlock;
  static const int nb = persistent_blocks(kernel, threads);
  const int want = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const int g = want < nb ? want : nb;
  *grid_out = g;
  hipLaunchKernelGGL(kernel, dim3((unsigned)g), dim3(threads), 0, st, a);
  return hipGetLastError();
}

// Tile depth along the marched axis: the deepest multiple of kUnroll (up to
// `cap`) that still yields enough wave tiles to fill the GPU; small levels
// get short tiles so that their march is short.
int tile_depth(int64_t columns, int n, int cap) {
  constexpr int64_t kWantTiles = 8192;
  int d = cap;
  while (d > kUnroll && columns * ((n + d - 1) / d) < kWantTiles) d -= kUnroll;
  return d;
}

}  // namespace

int classify_max_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess)
    cus = 256;
  return cus * 8;
}

void plan_level3(LevelDesc &l) {
  l.ntx = (l.mx + 63) / 64;
  l.nty = (l.my + kTile3Y - 1) / kTile3Y;
  l.zchunk = tile_depth((int64_t)l.ntx * l.nty, l.mz, kZChunk3);
  l.ntiles = l.ntx * l.nty * ((l.mz + l.zchunk - 1) / l.zchunk);
}

void plan_level2(LevelDesc &l) {
  l.ntx = (l.mx + 63) / 64;
  l.nty = 1;
  l.zchunk = tile_depth(l.ntx, l.my, kYChunk2);
  l.ntiles = l.ntx * ((l.my + l.zchunk - 1) / l.zchunk);
}

hipError_t launch_classify(const ClassifyArgs &a, int dim, bool read_prev,
                           bool write_masks, hipStream_t st, int *grid_out) {
  // fused launches compute the previous level's masks from the field
  const bool fused = a.nl > 1;
  if (dim == 3) {
    if (fused)
      return launch_persistent(classify3d_kernel<false, true, true>, a, st, grid_out);
    if (read_prev && write_masks)
      return launch_persistent(classify3d_kernel<true, true, false>, a, st, grid_out);
    if (read_prev)
      return launch_persistent(classify3d_kernel<true, false, false>, a, st, grid_out);
    if (write_masks)
      return launch_persistent(classify3d_kernel<false, true, false>, a, st, grid_out);
    return launch_persistent(classify3d_kernel<false, false, false>, a, st, grid_out);
  }
  if (fused)
    return launch_persistent(classify2d_kernel<false, true, true>, a, st, grid_out);
  if (read_prev && write_masks)
    return launch_persistent(classify2d_kernel<true, true, false>, a, st, grid_out);
  if (read_prev)
    return launch_persistent(classify2d_kernel<true, false, false>, a, st, grid_out);
  if (write_masks)
    return launch_persistent(classify2d_kernel<false, true, false>, a, st, grid_out);
  return launch_persistent(classify2d_kernel<false, false, false>, a, st, grid_out);
}

hipError_t launch_compact(const CompactArgs &a, bool fused, hipStream_t st) {
  if (a.nchunks > 1) {
    if (fused)
      hipLaunchKernelGGL(count_kernel<kFusedWordsPerThread>, dim3((unsigned)a.nchunks),
                         dim3(kCompactThreads), 0, st, a);
    else
      hipLaunchKernelGGL(count_kernel<kCompactWordsPerThread>,
                         dim3((unsigned)a.nchunks), dim3(kCompactThreads), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (fused)
    hipLaunchKernelGGL(expand_kernel<kFusedWordsPerThread>, dim3((unsigned)a.nchunks),
                       dim3(kCompactThreads), 0, st, a);
  else
    hipLaunchKernelGGL(expand_kernel<kCompactWordsPerThread>,
                       dim3((unsigned)a.nchunks), dim3(kCompactThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace pcrit
