// Classification and compaction kernels for gfx950 (MI355X).
//
// classify3d / classify2d: per-vertex critical-point classification of one
// level of the hierarchy, or of several small levels in one launch (wave
// tiles marched along the slowest axis, see below); the result per vertex is
// a code byte and a bit of the level's critical bitmask.
//
// count/expand: turn the per-level critical bitmask into the ascending list
// of full-resolution indices; the expansion is wave-cooperative, so every
// store instruction writes consecutive list entries.
#include <type_traits>
#include <utility>

#include "batch_tune.h"
#include "device_util.h"
#include "pcrit_internal.h"

// v_writelane: write a wave-uniform value into one lane of a register (the
// LLVM intrinsic, bound by name).
extern "C" __device__ int pcrit_writelane(int value, int lane, int old)
    __asm("llvm.amdgcn.writelane.i32");

namespace pcrit {
namespace {

using namespace dev;

// Boundary vertex with absent-neighbour mask A != 0 and raw mask mr (the
// table is indexed by raw masks, true mask = raw ^ kPos).  The link in the
// domain is the part of the full neighbour link spanned by the present
// neighbours.  Forcing the absent ones to "upper" leaves the lower link as
// the 0-bits; the 1-bits are then the complement of the lower link in the
// full link sphere, whose component count minus one is the lower link's
// number of holes (Alexander duality on the 2-sphere).  Symmetrically for
// the upper link with the absent neighbours forced to "lower".
__device__ __forceinline__ unsigned boundary_code3(const uint8_t *lut,
                                                   unsigned mr, unsigned A) {
  const unsigned eL = lut[(mr & ~A) | (~kPos3 & A)];  // true mask | A
  const unsigned eU = lut[(mr & ~A) | (kPos3 & A)];   // true mask & ~A
  const unsigned holes = ((eL >> 3) > 1u) | ((eU & 7u) > 1u);
  return (eL & 7u) | (eU & 0x38u) | 0x40u | (holes << 7);
}

// In 2D the link is a path at the boundary: its parts never have holes.
__device__ __forceinline__ unsigned boundary_code2(const uint8_t *lut,
                                                   unsigned mr, unsigned A) {
  return (lut[(mr & ~A) | (~kPos2 & A)] & 7u) |
         (lut[(mr & ~A) | (kPos2 & A)] & 0x38u) | 0x40u;
}

// Polarity masks by exact comparison.  Bit j is 1 iff neighbour j comes
// after the centre c in the order (value, full-resolution index).  For a
// neighbour with a larger index ("positive" offset: first non-zero of
// (dz, dy, dx) > 0) that is f >= c, for one with a smaller index f > c.
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
//   (3D) or a run of rows (2D), marched along the slowest axis.  The
//   columns left and right of the tile come from one packed halo load per
//   plane (row) and are shifted in at lanes 0 and 63.  The waves of a block
//   share only the link-pattern table, so there is no block barrier inside
//   the march.
// * The samples of the planes (rows) around the current one stay in
//   registers.  x-1 and x+1 neighbours are read from the lanes next door by
//   DPP wave shifts.
// * A polarity bit is the sign of one float difference, appended to the mask
//   with one alignbit.  For a centre c that is finite and non-zero the sign
//   of c - n (or n - c) is exact, ties included; a step in which some lane's
//   centre is +-0, +-inf or NaN recomputes its masks by exact comparisons.
// * Loads use a scalar plane (row) base and a 32-bit lane offset.  The march
//   issues loads only: on this architecture loads and stores share one
//   completion counter, and with a store in flight the compiler can no
//   longer wait for one particular load, so codes and masks are staged in
//   LDS (row-major) and written after the tile, several columns per lane.
// * A launch gives every wave one or two tiles; the tiles of one XCD form a
//   contiguous run, so neighbouring tiles (which share halo rows) meet in the
//   same L2.  A launch may cover several small levels (the progressive
//   driver fuses the latency-bound coarse levels); a wave then looks up the
//   level of its tile in the launch's level table.

// Level-(k+1) raw polarity mask of an old vertex, from its neighbours two
// level-k steps away (for levels classified in the same launch as the
// previous one, whose masks are then not stored).  Positions off the grid
// are clamped: their bits are masked by the caller.  (3D: inside the tile
// march.)
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
  return mask2(c, v) ^ kPos2;
}

// Absent-neighbour bits along x of column x on a level of mx columns.
__device__ __forceinline__ unsigned absent_x3(int x, int mx) {
  return (x == 0 ? AXM3 : 0u) | (x == mx - 1 ? AXP3 : 0u);
}
__device__ __forceinline__ unsigned absent_yz3(int y, int z, int my, int mz) {
  return (y == 0 ? AYM3 : 0u) | (y == my - 1 ? AYP3 : 0u) |
         (z == 0 ? AZM3 : 0u) | (z == mz - 1 ? AZP3 : 0u);
}
__device__ __forceinline__ unsigned absent_x2(int x, int mx) {
  return (x == 0 ? AXM2 : 0u) | (x == mx - 1 ? AXP2 : 0u);
}
__device__ __forceinline__ unsigned absent_y2(int y, int my) {
  return (y == 0 ? AYM2 : 0u) | (y == my - 1 ? AYP2 : 0u);
}
// Last coordinate of the next coarser level, in this level's steps.
__device__ __forceinline__ int coarse_last(int m) { return 2 * ((m - 1) >> 1); }

// ---------------------------------------------------------------------------
// 3D: one wave tile (64 columns x R rows x zchunk planes) of level g.
//   RP:  the previous level's masks are stored (g.prev_masks)
//   WM:  the level's masks may be stored for the next level (g.masks)
//   FAR: the previous level's masks may be computed from the field
// stc / stm: this wave's LDS staging for codes / masks.
// ---------------------------------------------------------------------------
template <int R>
struct Plane3 {
  float v[R + 2];      // rows y0-1 .. y0+R at this lane's column
  float hp;            // packed halo: lane i holds column x0-1 of row i,
                       // lane 64-NR+i column x0+64 of row i (i < NR)
  float l[R + 1];      // x-1 neighbour of rows 0..R
  float r[R + 1];      // x+1 neighbour of rows 1..R+1 (r[k]: row k+1)
  unsigned pm[R / 2];  // stored previous-level raw masks, even rows (even planes)
};

// Halo of row i from a packed halo register: lane 0 receives lane i (left
// halo), lane 63 receives lane 64-NR+i (right halo); row shifts within the
// 16-lane DPP rows.
template <int I>
__device__ __forceinline__ float halo_left(float hp) {
  if (I == 0) return hp;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(hp), 0x100 + I, 0xF, 0xF, false));
}
template <int I, int NR>
__device__ __forceinline__ float halo_right(float hp) {
  if (I == NR - 1) return hp;
  return __int_as_float(
      __builtin_amdgcn_mov_dpp(__float_as_int(hp), 0x110 + (NR - 1 - I), 0xF, 0xF, false));
}

// Tile classes: every vertex of a tile of class 1 or 2 is interior in y
// and z at its level and at the previous one, so the march needs no
// boundary logic except, in class 2, for the lanes at an x boundary; other
// tiles (class 0) take the general path.
template <int R>
__device__ __forceinline__ int tile_class3(const LevelDesc &g, int t) {
  const TilePos p = tile_pos(g, t);
  const int x0 = p.tx * kTileCols, y0 = p.ty * R, z0 = p.zc * g.zchunk;
  const int z1 = min(z0 + g.zchunk, g.mz);
  const bool y_in = y0 >= 1 && y0 + R <= min(g.my - 1, coarse_last(g.my));
  const bool z_in = z0 >= 1 && z1 <= min(g.mz - 1, coarse_last(g.mz));
  const bool x_in = x0 > 0 && x0 + kTileCols < min(g.mx, coarse_last(g.mx) + 1);
  return (y_in && z_in) ? (x_in ? 1 : 2) : 0;
}

template <int R, int ZC, bool RP, bool WM, bool FAR, int MODE>
__device__ __forceinline__ void tile3d(const ClassifyArgs &a,
                                       const LevelDesc &g, int t, int lane,
                                       const uint8_t *slut, uint8_t *stc,
                                       uint16_t *stm, bool &nan_seen,
                                       unsigned &reclass) {
  constexpr int NR = R + 2;
  constexpr int U = kUnroll3;  // ring of planes z-1 .. z+U-2
  static_assert(U >= 4 && U % 2 == 0 && R % 2 == 0, "plane ring and row parity");
  const int mx = g.mx, my = g.my, mz = g.mz;
  const TilePos tp = tile_pos(g, t);
  const int tx = tp.tx, ty = tp.ty, zc = tp.zc;
  const int x0 = tx * kTileCols;  // first column of the tile
  const int x = x0 + lane;        // this lane's column
  const int y0 = ty * R, z0 = zc * g.zchunk;  // both even
  const int z1 = min(z0 + g.zchunk, mz);
  const bool out_lane = x < mx;
  const uint64_t out_lanes = wave_ballot(out_lane);
  const uint64_t old_lanes = wave_ballot(out_lane && !(x & 1));
  const bool x_inner = x0 > 0 && x0 + kTileCols < mx;
  const bool dirty_test = (RP || FAR) && g.dirty;
  const bool store_masks = WM && g.masks != nullptr;
  const unsigned xA = absent_x3(x, mx);
  const int exc = coarse_last(mx), eyc = coarse_last(my), ezc = coarse_last(mz);
  const unsigned xA2 = (x == 0 ? AXM3 : 0u) | (x == exc ? AXP3 : 0u);

  // Loads: a buffer resource per plane, a 32-bit lane offset per row (a
  // plane is < 4 GiB).  One packed halo load per plane fetches the columns
  // left and right of the tile for all rows (clamped: a clamped sample is
  // never used).
  static_assert(NR <= 16, "packed halo within one DPP row");
  const int xc = min(x, mx - 1);
  const char *fb = reinterpret_cast<const char *>(g.f);
  const int64_t szb = g.sz * 4;
  uint32_t voff[NR];
#pragma unroll
  for (int i = 0; i < NR; i++)
    voff[i] = (uint32_t)(((int64_t)min(max(y0 - 1 + i, 0), my - 1) * g.sy +
                          (int64_t)xc * g.sx) * 4);
  uint32_t hpoff;
  {
    const bool left = lane < 32;
    const int hi = left ? min(lane, NR - 1) : max(lane - (64 - NR), 0);
    const int hx = left ? max(x0 - 1, 0) : min(x0 + 64, mx - 1);
    hpoff = (uint32_t)(((int64_t)min(max(y0 - 1 + hi, 0), my - 1) * g.sy +
                        (int64_t)hx * g.sx) * 4);
  }
  const char *pmb = reinterpret_cast<const char *>(g.prev_masks);
  const int64_t pmplane = (int64_t)g.pmx * g.pmy * 2;
  uint32_t pmoff[R / 2];
  if (RP) {
    const int pxc = min(xc >> 1, g.pmx - 1);
#pragma unroll
    for (int k = 0; k < R / 2; k++)
      pmoff[k] = (uint32_t)(((int64_t)min((y0 >> 1) + k, g.pmy - 1) * g.pmx + pxc) * 2);
  }
  // x offsets of the previous level's neighbours x-2, x, x+2 (clamped: the
  // bits of absent neighbours are masked by the dirty test)
  uint32_t fxo[FAR ? 3 : 1];
  if (FAR) {
#pragma unroll
    for (int d = 0; d < 3; d++)
      fxo[d] = (uint32_t)((int64_t)min(max(xc + 2 * (d - 1), 0), mx - 1) * g.sx * 4);
  }
  // plane z of the field / of the previous level's masks, z clamped
  auto plane_at = [&](int z) { return fb + (int64_t)min(max(z, 0), mz - 1) * szb; };
  // Previous-level raw mask of the old vertices of row (y, z), centre c:
  // its neighbours two level steps away, one buffer load each (plane base
  // and row offset scalar, column offset per lane), bits by the sign of the
  // difference as in the march (exact comparisons for special centres).
  auto far_mask = [&](int y, int z, float c) __attribute__((always_inline)) {
    float v[14];
#pragma unroll
    for (int j = 0; j < 14; j++) {
      const int dx = kOff3[j][0], dy = kOff3[j][1], dz = kOff3[j][2];
      const __amdgpu_buffer_rsrc_t r = rsrc(plane_at(z + 2 * dz));
      const int yy = min(max(y + 2 * dy, 0), my - 1);
      v[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          r, fxo[dx + 1], (int)((int64_t)yy * g.sy * 4), 0));
    }
    unsigned m = 0;
#pragma unroll
    for (int j = 13; j >= 0; j--)
      m = push_sign(m, ((kPos3 >> j) & 1u) ? v[j] - c : c - v[j]);
    if (wave_ballot(special_centre(c))) {
      const float lo[4] = {v[0], v[1], v[2], v[3]};
      const float md[6] = {v[4], v[5], v[6], v[7], v[8], v[9]};
      const float hi[4] = {v[10], v[11], v[12], v[13]};
      if (special_centre(c)) m = mask3(c, lo, md, hi) ^ kPos3;
    }
    return m;
  };
  auto pmplane_at = [&](int z) {
    return pmb + (int64_t)(min(max(z, 0), mz - 1) >> 1) * pmplane;
  };
  auto load = [&](const char *pp, const char *pmp, bool even, Plane3<R> &d) {
    const __amdgpu_buffer_rsrc_t r = rsrc(pp);
#pragma unroll
    for (int i = 0; i < NR; i++) d.v[i] = ld_f32(r, voff[i]);
    d.hp = ld_f32(r, hpoff);
    if (RP && even) {
      const __amdgpu_buffer_rsrc_t mr = rsrc(pmp);
#pragma unroll
      for (int k = 0; k < R / 2; k++) d.pm[k] = ld_u16(mr, pmoff[k]);
    }
  };
  // x-1 / x+1 neighbours of a loaded plane (lane shifts, halo at the ends)
  auto derive = [&](Plane3<R> &d) {
    static_for<R + 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      d.l[i] = shift_left(halo_left<i>(d.hp), d.v[i]);
    });
    static_for<R + 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value + 1;
      d.r[i - 1] = shift_right(halo_right<i, NR>(d.hp), d.v[i]);
    });
  };

  // lanes at an x boundary of this level or the previous one (class 2)
  const uint64_t xb_lanes = wave_ballot(out_lane && (xA | xA2) != 0u);

  unsigned wlo = 0, whi = 0;  // lane q: critical word of staged row q

  // Classify the R vertices of plane z (parity `even`) in this lane's column;
  // their staged rows start at qb.
  // Step of plane z: the bits from planes z-1 and z first, then the x-shifts
  // of plane z+1 (its loads were issued one step earlier: waiting for them
  // as late as possible), then the bits from plane z+1.
  auto step = [&](int z, bool even, int qb, const Plane3<R> &lo,
                  const Plane3<R> &mid, Plane3<R> &hi) {
    const bool zlive = z < z1;
    const bool z_inner = z > 0 && z < mz - 1;
    unsigned mr[R];
#pragma unroll
    for (int j = 0; j < R; j++) {
      const int i = j + 1;
      const float c = mid.v[i];
      unsigned m;
      m = push_sign(0u, mid.r[i] - c);             //  9 (1,1,0)
      m = push_sign(m, c - mid.l[i - 1]);          //  8 (-1,-1,0)
      m = push_sign(m, mid.v[i + 1] - c);          //  7 (0,1,0)
      m = push_sign(m, c - mid.v[i - 1]);          //  6 (0,-1,0)
      m = push_sign(m, mid.r[i - 1] - c);          //  5 (1,0,0)
      m = push_sign(m, c - mid.l[i]);              //  4 (-1,0,0)
      m = push_sign(m, c - lo.l[i - 1]);           //  3 (-1,-1,-1)
      m = push_sign(m, c - lo.v[i - 1]);           //  2 (0,-1,-1)
      m = push_sign(m, c - lo.l[i]);               //  1 (-1,0,-1)
      m = push_sign(m, c - lo.v[i]);               //  0 (0,0,-1)
      mr[j] = m;
    }
    derive(hi);
#pragma unroll
    for (int j = 0; j < R; j++) {
      const int i = j + 1;
      const float c = mid.v[i];
      unsigned m;
      m = push_sign(0u, hi.r[i] - c);              // 13 (1,1,1)
      m = push_sign(m, hi.v[i + 1] - c);           // 12 (0,1,1)
      m = push_sign(m, hi.r[i - 1] - c);           // 11 (1,0,1)
      m = push_sign(m, hi.v[i] - c);               // 10 (0,0,1)
      mr[j] |= m << 10;
    }
    // Rare: a centre whose differences may not carry the order.
    bool sp = false;
#pragma unroll
    for (int j = 0; j < R; j++) sp |= special_centre(mid.v[j + 1]);
    if (wave_ballot(sp)) {
#pragma unroll
      for (int j = 0; j < R; j++) {
        const int i = j + 1;
        const float c = mid.v[i];
        const float lov[4] = {lo.v[i], lo.l[i], lo.v[i - 1], lo.l[i - 1]};
        const float midv[6] = {mid.l[i],     mid.r[i - 1], mid.v[i - 1],
                               mid.v[i + 1], mid.l[i - 1], mid.r[i]};
        const float hiv[4] = {hi.v[i], hi.r[i - 1], hi.v[i + 1], hi.r[i]};
        const unsigned ex = mask3(c, lov, midv, hiv) ^ kPos3;
        mr[j] = special_centre(c) ? ex : mr[j];
        nan_seen |= zlive && y0 + j < my && out_lane && (c != c);
      }
    }
    // Per row: code, critical bit, dirty test.  IN: the tile is interior in
    // y and z at both levels (only x-boundary lanes differ).
    auto rows = [&](auto in_tag) __attribute__((always_inline)) {
      constexpr bool IN = decltype(in_tag)::value;
#pragma unroll
      for (int j = 0; j < R; j++) {
        const int y = y0 + j;
        unsigned code;
        uint64_t crit;
        if (IN) {
          code = slut[mr[j]];
          if (MODE == 2) {
            if (lane_bit(xb_lanes) && xA != 0u) code = boundary_code3(slut, mr[j], xA);
            crit = wave_ballot((code & 0xBFu) != 0x09u);
          } else {
            crit = wave_ballot(code != 0x09u);
          }
        } else {
          const bool inner = x_inner && z_inner && y > 0 && y < my - 1;
          if (inner) {
            code = slut[mr[j]];
            crit = wave_ballot(code != 0x09u);
          } else {
            const unsigned A = xA | absent_yz3(y, z, my, mz);
            code = A != 0u ? boundary_code3(slut, mr[j], A) : (unsigned)slut[mr[j]];
            crit = wave_ballot((code & 0xBFu) != 0x09u);
          }
        }
        unsigned out = code;
        if ((RP || FAR) && even && !(j & 1) && dirty_test) {
          // old vertex (present at level k+1): re-classified only if its
          // polarity mask or its set of absent neighbours changed
          unsigned pm = 0;
          if (RP) pm = mid.pm[j >> 1];
          if (FAR && !RP && out_lane && !(x & 1))
            pm = far_mask(y, z, mid.v[j + 1]);
          bool d;
          if (IN) {
            d = mr[j] != pm;  // both are 14-bit masks
            if (MODE == 2 && lane_bit(xb_lanes))
              d = xA2 != xA || ((mr[j] ^ pm) & ~xA & 0x3FFFu) != 0u;
          } else {
            const unsigned Af = xA | absent_yz3(y, z, my, mz);
            const unsigned A2 = xA2 | (y == 0 ? AYM3 : 0u) | (y == eyc ? AYP3 : 0u) |
                                (z == 0 ? AZM3 : 0u) | (z == ezc ? AZP3 : 0u);
            d = A2 != Af || ((mr[j] ^ pm) & ~Af & 0x3FFFu) != 0u;
          }
          const uint64_t old = (zlive && y < my) ? old_lanes : 0ull;
          const uint64_t dm = wave_ballot(d) & old;
          reclass += (unsigned)__popcll(dm);
        }
        const int q = qb + j;
        stc[q * 64 + lane] = (uint8_t)out;
        if (WM && store_masks) stm[q * 64 + lane] = (uint16_t)mr[j];
        wlo = (unsigned)pcrit_writelane((int)crit, q, (int)wlo);
        whi = (unsigned)pcrit_writelane((int)(crit >> 32), q, (int)whi);
      }
    };
    rows(std::integral_constant<bool, MODE != 0>{});
  };

  // Prologue: planes z0-1 .. z0+U-3 in flight; plane z sits in slot
  // (z - z0 + 1) % U, and step z loads plane z+U-2 into the slot of z-2.
  Plane3<R> W[U];
#pragma unroll
  for (int s = 0; s < U - 1; s++) {
    const int zs = min(z0 - 1 + s, z1);
    load(plane_at(zs), pmplane_at(zs), (s & 1) != 0, W[s]);
  }
  derive(W[0]);
  derive(W[1]);
  // running pointers to plane zn = z+U-2, clamped to plane z1 (the last one
  // the tile reads: the plane above its last classified plane) so that the
  // steps past the tile re-read a plane in cache instead of the next tile's
  const int zlast = min(z1, mz - 1);
  const char *pn = plane_at(min(z0 + U - 2, zlast));
  const char *pmn = pmplane_at(min(z0 + U - 2, zlast));
  int zn = z0 + U - 2;
  // zchunk is a multiple of U; a short last tile runs up to U-1 extra steps
  // whose staged rows are never written out.
  for (int zb = z0; zb < z1; zb += U) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int z = zb + u;
      load(pn, pmn, !(u & 1), W[(u + U - 1) % U]);
      if (zn < zlast) {
        pn += szb;
        if (u & 1) pmn += pmplane;  // plane zn+1 is even
      }
      zn++;
      step(z, !(u & 1), (z - z0) * R, W[u % U], W[(u + 1) % U], W[(u + 2) % U]);
    }
  }

  // Write the staged tile: per row a buffer resource at the row's start and
  // the lane's offset.
  const int nrows = (z1 - z0) * R;
  const uint64_t wbits = (((uint64_t)whi << 32) | wlo) & out_lanes;
  {
    const int q = lane;
    const int y = y0 + q % R, z = z0 + q / R;
    if (q < nrows && y < my)
      g.bits[((int64_t)z * my + y) * g.rowwords + tx] = wbits;
  }
  // rows per plane that exist (the last row tile may stick out)
  const int nyl = min(R, my - y0);
  const int nzl = z1 - z0;
  constexpr int NQ = ZC * R;
  // the flush reads staged rows that other lanes of this wave wrote
  wave_lds_sync();
  const bool full_tile = x0 + 64 <= mx && nyl == R;  // wave-uniform
  if (g.write_codes && g.sx == 1 && full_tile) {
    // Codes are staged row-major (row q at stc[64 q]): one dword per lane
    // covers four columns, a wave four rows, so each store instruction
    // writes four 64-byte row segments.
    const uint32_t *sp = reinterpret_cast<const uint32_t *>(stc);
    static_assert(64 % R == 0, "a dword group of staged rows spans whole planes");
    constexpr int PG = 4 / R;  // planes per group of four staged rows
    // lane offset within a group: plane, row, four columns (< 4 GiB: a
    // plane of codes is < 4 GiB and a group spans at most four rows)
    const int qs = lane >> 4;
    const uint32_t loff = (uint32_t)((qs / R) * g.sz + (qs % R) * g.sy) + 4u * (lane & 15);
    const uint8_t *cb = g.codes + (int64_t)z0 * g.sz + (int64_t)y0 * g.sy + x0;
#pragma unroll 4
    for (int k = 0; k < NQ / 4; k++) {
      if (k * PG >= nzl) break;
      const uint32_t v = sp[k * 64 + lane];
      if (PG * k + qs / R < nzl)
        __builtin_amdgcn_raw_buffer_store_b32(v, rsrc(cb + (int64_t)(PG * k) * g.sz), loff, 0, 0);
    }
  }
  if (!out_lane) return;
  // Strided levels, partial tiles and dense level codes: one byte per lane
  // and row, in a loop that is not unrolled (these are the rare paths; an
  // unrolled one would hoist every staged read into its own register).
  if ((g.write_codes && !(g.sx == 1 && full_tile)) || g.lcodes) {
    const bool full_res = g.write_codes && !(g.sx == 1 && full_tile);
    const uint32_t xoffc = (uint32_t)((int64_t)x * g.sx);
#pragma unroll 1
    for (int zz = 0; zz < nzl; zz++) {
#pragma unroll 1
      for (int j = 0; j < nyl; j++) {
        const unsigned b = stc[(zz * R + j) * 64 + lane];
        if (full_res)
          st_u8(rsrc(g.codes + (int64_t)(z0 + zz) * g.sz + (int64_t)(y0 + j) * g.sy), xoffc, b);
        if (g.lcodes)
          st_u8(rsrc(g.lcodes + ((int64_t)(z0 + zz) * my + (y0 + j)) * mx), (uint32_t)x, b);
      }
    }
  }
  if (WM && store_masks) {
    // Masks are staged row-major (row q at stm[64 q]).  Whole tiles of a
    // level with an even row length: one dword per lane covers two columns,
    // a wave two rows of one plane; otherwise one u16 per lane and row.
    char *mb = reinterpret_cast<char *>(g.masks);
    if (full_tile && !(mx & 1)) {
      static_assert(R == 2, "a dword group of staged mask rows is one plane");
      const uint32_t *sp = reinterpret_cast<const uint32_t *>(stm);
      const uint32_t loff = (uint32_t)((lane >> 5) * mx * 2) + 4u * (lane & 31);
      const char *pb = mb + (((int64_t)z0 * my + y0) * mx + x0) * 2;
      const int64_t mplane = (int64_t)my * mx * 2;
#pragma unroll 4
      for (int zz = 0; zz < ZC; zz++) {
        if (zz >= nzl) break;
        __builtin_amdgcn_raw_buffer_store_b32(sp[zz * 64 + lane], rsrc(pb + zz * mplane), loff, 0, 0);
      }
    } else if (out_lane) {
#pragma unroll 1
      for (int zz = 0; zz < nzl; zz++) {
#pragma unroll 1
        for (int j = 0; j < nyl; j++)
          st_u16(rsrc(mb + (((int64_t)(z0 + zz) * my + (y0 + j)) * mx) * 2), (uint32_t)x * 2u,
                 stm[(zz * R + j) * 64 + lane]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 2D: one wave tile (64 columns x zchunk rows) of level g, marched along y.
// ---------------------------------------------------------------------------
struct Row2 {
  float v, h;   // sample; as loaded, lane 0: x0-1, lane 63: x0+64
  float l, r;   // x-1 / x+1 neighbours
  unsigned pm;  // stored previous-level raw mask (even rows)
};

__device__ __forceinline__ int tile_class2(const LevelDesc &g, int t) {
  const TilePos p = tile_pos(g, t);  // 2D: one tile row, chunks along y
  const int x0 = p.tx * kTileCols, y0 = p.zc * g.zchunk;
  const int y1 = min(y0 + g.zchunk, g.my);
  const bool y_in = y0 >= 1 && y1 <= min(g.my - 1, coarse_last(g.my));
  const bool x_in = x0 > 0 && x0 + kTileCols < min(g.mx, coarse_last(g.mx) + 1);
  return y_in ? (x_in ? 1 : 2) : 0;
}

template <bool RP, bool WM, bool FAR, int MODE>
__device__ __forceinline__ void tile2d(const ClassifyArgs &a,
                                       const LevelDesc &g, int t, int lane,
                                       const uint8_t *slut, uint8_t *stc,
                                       uint8_t *stm, bool &nan_seen,
                                       unsigned &reclass) {
  constexpr int U = kUnroll2;  // ring of rows y-1 .. y+U-2
  static_assert(U % 2 == 0 && U >= 6, "row ring and row parity");
  const int mx = g.mx, my = g.my;
  const TilePos tp = tile_pos(g, t);  // 2D: one tile row, chunks along y
  const int tx = tp.tx, yc = tp.zc;
  const int x0 = tx * kTileCols;
  const int x = x0 + lane;
  const int y0 = yc * g.zchunk;  // even
  const int y1 = min(y0 + g.zchunk, my);
  const bool out_lane = x < mx;
  const uint64_t out_lanes = wave_ballot(out_lane);
  const uint64_t old_lanes = wave_ballot(out_lane && !(x & 1));
  const bool x_inner = x0 > 0 && x0 + kTileCols < mx;
  const bool dirty_test = (RP || FAR) && g.dirty;
  const bool store_masks = WM && g.masks != nullptr;
  const unsigned xA = absent_x2(x, mx);
  const int exc = coarse_last(mx), eyc = coarse_last(my);
  const unsigned xA2 = (x == 0 ? AXM2 : 0u) | (x == exc ? AXP2 : 0u);
  const uint64_t xb_lanes = wave_ballot(out_lane && (xA | xA2) != 0u);
  const int xc = min(x, mx - 1);
  const int xh = lane == 0 ? max(x0 - 1, 0) : (lane == 63 ? min(x0 + 64, mx - 1) : xc);
  const uint32_t xoff = (uint32_t)((int64_t)xc * g.sx * 4);
  const uint32_t hoff = (uint32_t)((int64_t)xh * g.sx * 4);
  const char *fb = reinterpret_cast<const char *>(g.f);
  const int64_t syb = g.sy * 4;
  const char *pmb = reinterpret_cast<const char *>(g.prev_masks);
  const uint32_t pmx_off = RP ? (uint32_t)min(xc >> 1, g.pmx - 1) : 0u;

  auto load = [&](int y, bool even, Row2 &d) {
    const int ycl = min(max(y, 0), my - 1);
    const __amdgpu_buffer_rsrc_t r = rsrc(fb + (int64_t)ycl * syb);
    d.v = ld_f32(r, xoff);
    d.h = ld_f32(r, hoff);
    if (RP && even)
      d.pm = ld_u8(rsrc(pmb + (int64_t)min(ycl >> 1, g.pmy - 1) * g.pmx), pmx_off);
  };
  auto derive = [&](Row2 &d) {
    d.l = shift_left(d.h, d.v);
    d.r = shift_right(d.h, d.v);
  };
  unsigned wlo = 0, whi = 0;

  auto step = [&](int y, bool even, const Row2 &lo, const Row2 &mid,
                  const Row2 &hi) {
    const float c = mid.v;
    unsigned m;
    m = push_sign(0u, hi.r - c);   // 5 (1,1)
    m = push_sign(m, c - lo.l);    // 4 (-1,-1)
    m = push_sign(m, hi.v - c);    // 3 (0,1)
    m = push_sign(m, c - lo.v);    // 2 (0,-1)
    m = push_sign(m, mid.r - c);   // 1 (1,0)
    m = push_sign(m, c - mid.l);   // 0 (-1,0)
    if (wave_ballot(special_centre(c))) {
      const float nb[6] = {mid.l, mid.r, lo.v, hi.v, lo.l, hi.r};
      const unsigned ex = mask2(c, nb) ^ kPos2;
      m = special_centre(c) ? ex : m;
      nan_seen |= y < y1 && out_lane && (c != c);
    }
    unsigned code;
    uint64_t crit;
    if (MODE != 0) {
      code = slut[m];
      if (MODE == 2) {
        if (lane_bit(xb_lanes) && xA != 0u) code = boundary_code2(slut, m, xA);
        crit = wave_ballot((code & 0xBFu) != 0x09u);
      } else {
        crit = wave_ballot(code != 0x09u);
      }
    } else if (x_inner && y > 0 && y < my - 1) {
      code = slut[m];
      crit = wave_ballot(code != 0x09u);
    } else {
      const unsigned A = xA | absent_y2(y, my);
      code = A != 0u ? boundary_code2(slut, m, A) : (unsigned)slut[m];
      crit = wave_ballot((code & 0xBFu) != 0x09u);
    }
    unsigned out = code;
    if ((RP || FAR) && even && dirty_test) {
      unsigned pm = 0;
      if (RP) pm = mid.pm;
      if (FAR && !RP && out_lane && !(x & 1)) pm = far_mask2(g.f, g, x, y, c);
      bool d;
      if (MODE != 0) {
        d = m != pm;  // both are 6-bit masks
        if (MODE == 2 && lane_bit(xb_lanes))
          d = xA2 != xA || ((m ^ pm) & ~xA & 0x3Fu) != 0u;
      } else {
        const unsigned Af = xA | absent_y2(y, my);
        const unsigned A2 = xA2 | (y == 0 ? AYM2 : 0u) | (y == eyc ? AYP2 : 0u);
        d = A2 != Af || ((m ^ pm) & ~Af & 0x3Fu) != 0u;
      }
      uint64_t dm = wave_ballot(d);
      const uint64_t old = y < y1 ? old_lanes : 0ull;
      dm &= old;
      reclass += (unsigned)__popcll(dm);
    }
    const int q = y - y0;
    stc[q * 64 + lane] = (uint8_t)out;
    if (WM && store_masks) stm[q * 64 + lane] = (uint8_t)m;
    wlo = (unsigned)pcrit_writelane((int)crit, q, (int)wlo);
    whi = (unsigned)pcrit_writelane((int)(crit >> 32), q, (int)whi);
  };

  // Row y sits in slot (y - y0 + 1) % U; step y loads row y + U - 2 into
  // the slot of row y-2.
  Row2 W[U];
#pragma unroll
  for (int s = 0; s < U - 1; s++) load(y0 - 1 + s, (s & 1) != 0, W[s]);
  derive(W[0]);
  derive(W[1]);
  for (int yb = y0; yb < y1; yb += U) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int y = yb + u;
      derive(W[(u + 2) % U]);  // row y+1
      load(y + U - 2, !(u & 1), W[(u + U - 1) % U]);
      step(y, !(u & 1), W[u % U], W[(u + 1) % U], W[(u + 2) % U]);
    }
  }

  const int nrows = y1 - y0;
  const uint64_t wbits = (((uint64_t)whi << 32) | wlo) & out_lanes;
  if (lane < nrows) g.bits[(int64_t)(y0 + lane) * g.rowwords + tx] = wbits;
  // Codes and masks are staged row-major (row q at 64 q).  Whole tiles with
  // aligned rows: one dword per lane covers four columns, a wave four rows;
  // otherwise one byte per lane and row in a rolled loop.
  wave_lds_sync();
  const bool full_tile = x0 + 64 <= mx;  // wave-uniform
  auto rows4 = [&](const uint8_t *st, uint8_t *base, int64_t rstride) {
    const uint32_t *sp = reinterpret_cast<const uint32_t *>(st);
    const int qs = lane >> 4;
    const uint32_t loff = (uint32_t)(qs * rstride) + 4u * (lane & 15);
#pragma unroll 4
    for (int k = 0; k < kYChunk2 / 4; k++) {
      if (4 * k >= nrows) break;
      const uint32_t v = sp[k * 64 + lane];
      if (4 * k + qs < nrows)
        __builtin_amdgcn_raw_buffer_store_b32(v, rsrc(base + (int64_t)(4 * k) * rstride),
                                              loff, 0, 0);
    }
  };
  const bool codes4 = g.write_codes && g.sx == 1 && full_tile && !(g.sy & 3);
  if (codes4) rows4(stc, g.codes + (int64_t)y0 * g.sy + x0, g.sy);
  const bool masks4 = WM && store_masks && full_tile && !(mx & 3);
  if (masks4) rows4(stm, reinterpret_cast<uint8_t *>(g.masks) + (int64_t)y0 * mx + x0, mx);
  if (!out_lane) return;
  const bool codes1 = g.write_codes && !codes4;
  const bool masks1 = WM && store_masks && !masks4;
  if (codes1 || masks1 || g.lcodes) {
    const uint32_t xoffc = (uint32_t)((int64_t)x * g.sx);
#pragma unroll 1
    for (int q = 0; q < nrows; q++) {
      const unsigned b = stc[q * 64 + lane];
      if (codes1) st_u8(rsrc(g.codes + (int64_t)(y0 + q) * g.sy), xoffc, b);
      if (g.lcodes) st_u8(rsrc(g.lcodes + (int64_t)(y0 + q) * mx), (uint32_t)x, b);
      if (masks1)
        st_u8(rsrc(reinterpret_cast<uint8_t *>(g.masks) + (int64_t)(y0 + q) * mx),
              (uint32_t)x, stm[q * 64 + lane]);
    }
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
  constexpr int ZC = zchunk_cap3(WM);
  static_assert(ZC % kUnroll3 == 0, "tile depth must be a multiple of the unroll");
  static_assert(ZC * R <= 64, "one critical word per lane");
  static_assert(ZC % 2 == 0, "mask staging in two halves");
  __shared__ __attribute__((aligned(16))) uint8_t slut[kLut3Size];
  __shared__ __attribute__((aligned(16))) uint8_t scode[NW][64 * ZC * R];
  __shared__ __attribute__((aligned(16))) uint16_t smask[WM ? NW : 1][WM ? 64 * ZC * R : 2];
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
    const LevelDesc &lv = a.lv[l];
    const int tt = t - lv.tile_begin;
    const int cls = tile_class3<R>(lv, tt);
    if (cls == 1)
      tile3d<R, ZC, RP, WM, FAR, 1>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                                nan_seen, reclass);
    else if (cls == 2)
      tile3d<R, ZC, RP, WM, FAR, 2>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                                nan_seen, reclass);
    else
      tile3d<R, ZC, RP, WM, FAR, 0>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                                nan_seen, reclass);
    if ((RP || FAR) && lane == 0 && reclass) atomicAdd(&s_reclass[l], reclass);
  }
  if (wave_ballot(nan_seen) && lane == 0) *a.nan_flag = a.gen;
  __syncthreads();
  if ((RP || FAR) && tid < a.nl && s_reclass[tid])
    atomicAdd(&a.reclass_acc[tid], s_reclass[tid]);
}

template <bool RP, bool WM, bool FAR>
__global__ __launch_bounds__(64 * kWavesPerBlock) void classify2d_kernel(
    ClassifyArgs a) {
  constexpr int NW = kWavesPerBlock;
  constexpr int YC = kYChunk2;
  static_assert(YC % kUnroll2 == 0 && YC <= 64, "tile depth");
  __shared__ uint8_t slut[kLut2Size];
  __shared__ __attribute__((aligned(16))) uint8_t scode[NW][64 * kYChunk2];
  __shared__ __attribute__((aligned(16))) uint8_t smask[WM ? NW : 1][WM ? 64 * kYChunk2 : 4];
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
    const LevelDesc &lv = a.lv[l];
    const int tt = t - lv.tile_begin;
    const int cls = tile_class2(lv, tt);
    if (cls == 1)
      tile2d<RP, WM, FAR, 1>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                             nan_seen, reclass);
    else if (cls == 2)
      tile2d<RP, WM, FAR, 2>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                             nan_seen, reclass);
    else
      tile2d<RP, WM, FAR, 0>(a, lv, tt, lane, slut, scode[w], smask[WM ? w : 0],
                             nan_seen, reclass);
    if ((RP || FAR) && lane == 0 && reclass) atomicAdd(&s_reclass[l], reclass);
  }
  if (wave_ballot(nan_seen) && lane == 0) *a.nan_flag = a.gen;
  __syncthreads();
  if ((RP || FAR) && tid < a.nl && s_reclass[tid])
    atomicAdd(&a.reclass_acc[tid], s_reclass[tid]);
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

// The list offsets of a call for the caller (device), the total -1 after a
// NaN sample.
__global__ __launch_bounds__(64) void publish_kernel(const int64_t *level_base, int n,
                                                     const unsigned *nan_flag,
                                                     unsigned gen, int64_t *out) {
  const int i = threadIdx.x;
  if (i < n) out[i] = (i == n - 1 && *nan_flag == gen) ? -1 : level_base[i];
}

// Inclusive prefix sum over the lanes of a wave: shifts within the 16-lane
// DPP rows, then the row broadcasts of lanes 15 and 31.  Lanes without a
// source add the `old` operand, 0.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// expand_kernel: every wave owns a contiguous run of WPT * 64 words of the
// chunk, loaded at once (one word per lane and round).  One block scan of
// the waves' popcount totals places each wave's run; after that the waves
// work on their own: in a round every lane expands its word into the wave's
// LDS region at its position (DPP scan of the popcounts) as 16-bit entries
// (word << 6 | bit), low half then high half, and the wave writes the
// round's entries to the list with coalesced stores.  Entries are in index
// order because words are in index order and bits are expanded low to high.
// On a linear level (full resolution, rows a whole number of words) the
// index of an entry is 64 * (first word of the round) + entry; otherwise it
// comes from the word's row start.
template <int WPT>
__global__ __launch_bounds__(kCompactThreads) void expand_kernel(CompactArgs a) {
  constexpr int T = kCompactThreads;
  constexpr int CW = T * WPT;
  constexpr int NWV = T / 64;
  __shared__ int64_t s_red[NWV];
  __shared__ int s_wtot[NWV];
  __shared__ uint16_t s_ent[NWV][64 * 64];
  __shared__ uint32_t s_row0[NWV][64];
  const int chunk = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = level_of_chunk(a, chunk);
  const CompactLevel &L = a.lv[li];
  const int lchunk = chunk - L.chunk_begin;
  // first word of this wave's run
  const int64_t wrun = (int64_t)lchunk * CW + (int64_t)w * (64 * WPT);
  uint64_t wd[WPT];
#pragma unroll
  for (int k = 0; k < WPT; k++) {
    const int64_t gw = wrun + (int64_t)k * 64 + lane;
    wd[k] = gw < L.words ? L.bits[gw] : 0ull;
  }

  // entries before this chunk, and before this chunk's level, in this launch
  int64_t part = 0, lpart = 0;
  {
    constexpr int U = 8;  // counts loaded per round, independent loads
    for (int i0 = 0; i0 < chunk; i0 += U * T) {
      int c[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int i = i0 + u * T + tid;
        c[u] = i < chunk ? a.counts[i] : 0;
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int i = i0 + u * T + tid;
        part += c[u];
        lpart += i < L.chunk_begin ? c[u] : 0;
      }
    }
  }
  const int64_t prefix = block_sum(part, s_red);
  const int64_t lprefix = block_sum(lpart, s_red);
  // lists of earlier launches end at level_base[first slot of this launch]
  const int64_t base = a.level_base[a.lv[0].slot];
  if (lchunk == 0 && tid == 0) {
    // the counter starts at zero for the next launch on this stream
    const unsigned r = a.reclass_acc[li];
    a.reclass_acc[li] = 0u;
    if (L.reclass_out) *L.reclass_out = r;
  }
  // this wave's place in the chunk
  int cnt_all = 0;
#pragma unroll
  for (int k = 0; k < WPT; k++) cnt_all += __popcll(wd[k]);
  const int wtot = __builtin_amdgcn_readlane(wave_inclusive_sum(cnt_all), 63);
  if (lane == 0) s_wtot[w] = wtot;
  __syncthreads();
  int woff = 0, ctot = 0;
#pragma unroll
  for (int i = 0; i < NWV; i++) {
    woff += i < w ? s_wtot[i] : 0;
    ctot += s_wtot[i];
  }

  const bool linear = L.linear && !a.crit_codes;
  const int64_t rowstep = L.s * L.nx;
  const uint32_t s = (uint32_t)L.s;
  uint16_t *went = s_ent[w];
  int64_t out0 = base + prefix + woff;  // list position of the round's first entry
#pragma unroll
  for (int k = 0; k < WPT; k++) {
    const int64_t gw0 = wrun + (int64_t)k * 64;  // first word of the round
    uint32_t lo = (uint32_t)wd[k], hi = (uint32_t)(wd[k] >> 32);
    const int cnt = __popc(lo) + __popc(hi);
    const int incl = wave_inclusive_sum(cnt);
    const int tot = __builtin_amdgcn_readlane(incl, 63);
    if (!linear && (lo | hi)) {
      // word gw covers columns 64*xw + bit of level row r
      const uint32_t gw = (uint32_t)(gw0 + lane);
      const uint32_t r = gw / (uint32_t)L.rowwords;
      const uint32_t xw = gw - r * (uint32_t)L.rowwords;
      const uint32_t zz = r / (uint32_t)L.my, yy = r - zz * (uint32_t)L.my;
      s_row0[w][lane] = (uint32_t)(rowstep * ((int64_t)yy + L.ny * (int64_t)zz) +
                                   L.s * (int64_t)xw * kTileCols);
    }
    {
      // low half, then high half, from this lane's position
      const unsigned e0 = (unsigned)lane << 6;
      uint16_t *ep = went + (incl - cnt);
      while (lo) {
        *ep++ = (uint16_t)(e0 | (unsigned)__builtin_ctz(lo));
        lo &= lo - 1u;
      }
      const unsigned e1 = e0 | 32u;
      while (hi) {
        *ep++ = (uint16_t)(e1 | (unsigned)__builtin_ctz(hi));
        hi &= hi - 1u;
      }
    }
    wave_lds_sync();
    // entries of this round that fit the capacity
    const int lim = (int)max((int64_t)0, min((int64_t)tot, a.cap - out0));
    uint32_t *dst = a.crit + out0;
    if (linear) {
      const uint32_t ibase = (uint32_t)(gw0 * 64);
      // whole groups of UW * 64 entries without bounds tests, then the tail
      constexpr int UW = 4;
      const int lim_full = lim - lim % (UW * 64);
      for (int e0 = 0; e0 < lim_full; e0 += UW * 64) {
        uint32_t v[UW];
#pragma unroll
        for (int u = 0; u < UW; u++) v[u] = went[e0 + u * 64 + lane];
#pragma unroll
        for (int u = 0; u < UW; u++) dst[e0 + u * 64 + lane] = ibase + v[u];
      }
      for (int e = lim_full + lane; e < lim; e += 64) dst[e] = ibase + went[e];
    } else {
      for (int e = lane; e < lim; e += 64) {
        const unsigned ent = went[e];
        const uint32_t idx = s_row0[w][ent >> 6] + s * (ent & 63u);
        dst[e] = idx;
        if (a.crit_codes) {
          uint8_t code;
          if (L.lcodes) {
            // dense level index from the full-resolution one
            const uint32_t xf = idx % (uint32_t)L.nx, rest = idx / (uint32_t)L.nx;
            const uint32_t yf = rest % (uint32_t)L.ny, zf = rest / (uint32_t)L.ny;
            const int64_t lix = ((int64_t)(zf / s) * L.my + yf / s) * L.mx + xf / s;
            code = L.lcodes[lix];
          } else {
            code = L.codes[idx];
          }
          a.crit_codes[out0 + e] = code;
        }
      }
    }
    out0 += tot;
    wave_lds_sync();  // the next round overwrites this wave's entries
  }

  // the first chunk of a later level opens its list, the last chunk of the
  // launch closes the last one
  if (li > 0 && lchunk == 0 && tid == 0) a.level_base[L.slot] = base + prefix;
  if (chunk == a.nchunks - 1 && tid == 0) {
    const int64_t total = prefix + ctot;
    a.level_base[L.slot + 1] = base + total;
    const bool nan = *a.nan_flag == a.gen;
    if (a.count_dev) *a.count_dev = nan ? -1 : total - lprefix;
    // single-level launch: every other list offset was written by an
    // earlier launch, the last one just above
    if (a.publish) {
      for (int i = 0; i + 1 < a.publish_n; i++) a.publish[i] = a.level_base[i];
      a.publish[a.publish_n - 1] = nan ? -1 : base + total;
    }
  }
}

// Grid of a classification launch: every wave takes kTileRounds tiles (the
// kernels stride over the tiles by the grid's wave count), one in fused
// launches of small levels, whose few tiles are latency bound.  Short blocks
// let the dispatcher balance tiles of unequal cost (boundary tiles, the
// re-classification branch) over the CUs better than a fixed persistent
// share per block does.
constexpr int kTileRounds = 2;

template <auto Kernel>
hipError_t launch_tiles(const ClassifyArgs &a, hipStream_t st) {
  const int threads = 64 * kWavesPerBlock;
  const int64_t per_block = (int64_t)kWavesPerBlock * (a.nl > 1 ? 1 : kTileRounds);
  const int g = (int)((a.ntiles + per_block - 1) / per_block);
  hipLaunchKernelGGL(Kernel, dim3((unsigned)(g > 0 ? g : 1)), dim3(threads), 0, st, a);
  return hipGetLastError();
}

// Tile depth along the marched axis: the deepest multiple of `step` (up to
// `cap`) that still yields `want` wave tiles; only levels too small for that
// get shorter tiles.  Fused launches of small levels aim at 2048 tiles (two
// per SIMD; aiming at 8192 made the fused coarse launch 36 instead of 30 us:
// more waves than fit at once, each with a short march).  Single-level
// launches aim at 8192 tiles, so that mid-size levels still spread over
// most resident wave slots (measured at level 0 of the smooth 256^3 field:
// 2048 tiles 47.6 us, 8192 tiles 39.9 us, 16384 45.0 us, 32768 61.8 us;
// the 512^3 levels have more tiles than any of these at full depth).
constexpr int64_t kWantTilesFused = 2048;
constexpr int64_t kWantTilesLevel = 8192;
int tile_depth(int64_t columns, int n, int cap, int step, int64_t want) {
  int d = cap;
  while (d > step && columns * ((n + d - 1) / d) < want) d -= step;
  return d;
}

}  // namespace

void plan_level3_want(LevelDesc &l, bool write_masks, int64_t want) {
  l.ntx = (l.mx + kTileCols - 1) / kTileCols;
  l.nty = (l.my + kTile3Y - 1) / kTile3Y;
  l.zchunk = tile_depth((int64_t)l.ntx * l.nty, l.mz, zchunk_cap3(write_masks), kUnroll3, want);
  l.ntiles = l.ntx * l.nty * ((l.mz + l.zchunk - 1) / l.zchunk);
  fast_divisor((uint32_t)l.ntx, &l.ntx_mul, &l.ntx_shift);
  fast_divisor((uint32_t)l.nty, &l.nty_mul, &l.nty_shift);
}

void plan_level2_want(LevelDesc &l, int64_t want) {
  l.ntx = (l.mx + kTileCols - 1) / kTileCols;
  l.nty = 1;
  l.zchunk = tile_depth(l.ntx, l.my, kYChunk2, kUnroll2, want);
  l.ntiles = l.ntx * ((l.my + l.zchunk - 1) / l.zchunk);
  fast_divisor((uint32_t)l.ntx, &l.ntx_mul, &l.ntx_shift);
  fast_divisor(1u, &l.nty_mul, &l.nty_shift);
}

void plan_level3(LevelDesc &l, bool write_masks, bool fused) {
  plan_level3_want(l, write_masks, fused ? kWantTilesFused : kWantTilesLevel);
}

void plan_level2(LevelDesc &l, bool fused) {
  plan_level2_want(l, fused ? kWantTilesFused : kWantTilesLevel);
}

hipError_t launch_classify(const ClassifyArgs &a, int dim, bool read_prev,
                           bool write_masks, bool fused, hipStream_t st) {
  // fused launches (several levels, or a batch of fields) compute an old
  // vertex's previous-level mask from the field when their level asks for it
  if (dim == 3) {
    // the kernel's LDS staging holds tiles of at most zchunk_cap3 planes
    for (int l = 0; l < a.nl; l++)
      if (a.lv[l].zchunk > zchunk_cap3(fused || write_masks)) return hipErrorInvalidValue;
    if (fused)
      return launch_tiles<classify3d_kernel<false, true, true>>(a, st);
    if (read_prev && write_masks)
      return launch_tiles<classify3d_kernel<true, true, false>>(a, st);
    if (read_prev)
      return launch_tiles<classify3d_kernel<true, false, false>>(a, st);
    if (write_masks)
      return launch_tiles<classify3d_kernel<false, true, false>>(a, st);
    return launch_tiles<classify3d_kernel<false, false, false>>(a, st);
  }
  if (fused)
    return launch_tiles<classify2d_kernel<false, true, true>>(a, st);
  if (read_prev && write_masks)
    return launch_tiles<classify2d_kernel<true, true, false>>(a, st);
  if (read_prev)
    return launch_tiles<classify2d_kernel<true, false, false>>(a, st);
  if (write_masks)
    return launch_tiles<classify2d_kernel<false, true, false>>(a, st);
  return launch_tiles<classify2d_kernel<false, false, false>>(a, st);
}

hipError_t launch_publish_offsets(const int64_t *level_base, int n,
                                  const unsigned *nan_flag, unsigned gen,
                                  int64_t *out, hipStream_t st) {
  if (n < 1 || n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(64), 0, st, level_base, n, nan_flag,
                     gen, out);
  return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs &a, bool small, hipStream_t st) {
  if (a.nchunks > 1) {
    if (small)
      hipLaunchKernelGGL(count_kernel<kSmallWordsPerThread>, dim3((unsigned)a.nchunks),
                         dim3(kCompactThreads), 0, st, a);
    else
      hipLaunchKernelGGL(count_kernel<kCompactWordsPerThread>,
                         dim3((unsigned)a.nchunks), dim3(kCompactThreads), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (small)
    hipLaunchKernelGGL(expand_kernel<kSmallWordsPerThread>, dim3((unsigned)a.nchunks),
                       dim3(kCompactThreads), 0, st, a);
  else
    hipLaunchKernelGGL(expand_kernel<kCompactWordsPerThread>,
                       dim3((unsigned)a.nchunks), dim3(kCompactThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace pcrit
