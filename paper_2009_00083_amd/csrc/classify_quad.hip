// Quad-tile classification of full-resolution and stride-2 levels of 3D
// grids (gfx950).
//
// A wave owns 256 consecutive level columns -- four per lane, read with one
// 16-byte load per row at full resolution (two at stride 2) -- by R rows,
// and marches them along z with three planes in registers (the current one,
// the next one, and the one after it in flight).
//
// Every edge of the triangulation is subtracted once.  For a vertex v the
// seven differences f(v + d) - f(v) towards its later neighbours (the
// offsets d with all components >= 0) give the sign bits P(v): bit j is 1
// iff neighbour v + d_j comes before v in the order (value, index) -- for
// finite, non-zero samples the sign of the float difference is exact, ties
// included.  The bits towards the earlier neighbours v - d_j are the same
// edge signs read from the P bytes of those neighbours: N(v) bit j is bit j
// of P(v - d_j), 1 iff v - d_j comes after v.  P and N are kept as bytes,
// four vertices per register, so N is assembled with one and-or per
// direction for four vertices, and P(v) | N(v) << 8 indexes a 32 KiB table
// in LDS that holds the code byte (lower and upper link component counts)
// of each polarity pattern.
//
// Boundary vertices force their absent neighbours (two table reads, as the
// other kernels do).  Centres whose differences may not carry the order
// (+-0, +-inf, NaN) are re-classified after the march by comparisons, which
// also report NaN samples.
//
// The critical bits of a row leave as the level's 64-bit bitmask words
// (bit b = column 64 w + b): each lane shifts its four bits to its place in
// a word and sixteen lanes OR them together with DPP row shifts.
#include <algorithm>

#include "device_util.h"
#include "pcrit_internal.h"

// v_writelane: write a wave-uniform value into one lane of a register.
extern "C" __device__ int pcrit_q_writelane(int value, int lane, int old)
    __asm("llvm.amdgcn.writelane.i32");

namespace pcrit {
namespace {

using namespace dev;

constexpr unsigned QAXM = quad_side(0, -1), QAXP = quad_side(0, 1);
constexpr unsigned QAYM = quad_side(1, -1), QAYP = quad_side(1, 1);
constexpr unsigned QAZM = quad_side(2, -1), QAZP = quad_side(2, 1);

// Buffer resource with a record limit: loads past it return zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_n(const void *base, uint32_t nrec) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)nrec,
                                           0x00020000);
}
// 16 bytes at lane offset voff + wave-uniform offset soff
__device__ __forceinline__ float4 ld128(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float old, float src) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                    CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u(unsigned old, unsigned src) {
  return (unsigned)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float mov_dpp_f(float src) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ unsigned mov_dpp_u(unsigned src) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)src, CTRL, 0xF, 0xF, false);
}
// m shifted up by 32 - s bits, the top 32 - s bits of d below
__device__ __forceinline__ unsigned push_bits(unsigned m, float d, int s) {
  return __builtin_amdgcn_alignbit(m, __float_as_uint(d), s);
}
// Boundary vertex: the absent neighbours (bits A of the quad index) forced
// to "upper" leave the lower link as the lower neighbours and its complement
// in the full link sphere; forced to "lower", the same for the upper link
// (holes from Alexander duality on the 2-sphere).
__device__ __forceinline__ unsigned quad_boundary(const uint8_t *lut, unsigned idx,
                                                  unsigned A) {
  const unsigned base = idx & ~A;
  const unsigned eL = lut[base | (A & kQNeg)];
  const unsigned eU = lut[base | (A & kQPos)];
  const unsigned holes = ((eL >> 3) > 1u) | ((eU & 7u) > 1u);
  return (eL & 7u) | (eU & 0x38u) | 0x40u | (holes << 7);
}

template <int R, int SX>
struct QPlane {
  // SX = 1: rows y0-1 .. y0+R, level columns c0 .. c0+3 of this lane.  SX =
  // 2: each row's eight samples as loaded (the level columns are the even
  // ones), kept as loaded so that no copy waits for the load
  float4 raw[SX][R + 2];
  float h;          // packed halo: lane i < R+2 column x0-1 of row i, lane
                    // 16+i column x0, lane 48+i column x0+256
  __device__ __forceinline__ float4 v(int i) const {
    if constexpr (SX == 1)
      return raw[0][i];
    else
      return make_float4(raw[0][i].x, raw[0][i].z, raw[1][i].x, raw[1][i].z);
  }
  // SX = 2: the odd samples are never read, so the compiler would hand their
  // registers to other values while the load is in flight and wait for it
  // there; an empty use just before the slot is loaded again keeps them
  __device__ __forceinline__ void keep() const {
    if constexpr (SX == 2) {
#pragma unroll
      for (int i = 0; i < R + 2; i++) asm volatile("" ::"v"(raw[0][i].y), "v"(raw[1][i].y));
    }
  }
};

// s_waitcnt operand: vmcnt 0, expcnt and lgkmcnt unconstrained (GFX9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVmem = 0x0F70;

// GEN: the tile has rows or planes on the y or z boundary of the level.
// CODES: the codes are stored (always at stride 1; at stride 2 a launch
// without a codes array, as in progressive calls without list codes, leaves
// the store instructions out).
template <int R, int SX, bool GEN, bool CODES>
__device__ __forceinline__ void quad_tile(const QuadArgs &a, int t, int lane,
                                          const uint8_t *slut, bool &nan_seen) {
  const LevelDesc &g = a.lv;
  constexpr int NR = R + 2;
  constexpr int NS = kQuadSlots;           // planes in registers: z .. z+NS-1
  constexpr int U = NS % 2 ? 2 * NS : NS;   // unroll: NS plane slots, two P slots
  static_assert(NR <= 16 && 4 * R <= 64, "packed halo in one DPP row, bit words in one wave");
  const int mx = g.mx, my = g.my, mz = g.mz;
  const TilePos tp = tile_pos(g, t);
  const int x0 = tp.tx * kQuadCols, y0 = tp.ty * R, z0 = tp.zc * g.zchunk;
  const int z1 = min(z0 + g.zchunk, mz);
  const int zlim = min(z1, mz - 1);  // last plane the tile reads
  const int c0 = x0 + 4 * lane;      // level column of this lane's first vertex
  const int nval = min(max(mx - c0, 0), 4);
  const bool full = x0 + kQuadCols <= mx;  // every lane holds four columns

  // Addresses: a buffer resource per plane (its record limit ends at the
  // field's end), 32-bit byte offsets within the plane.  Lanes past the
  // last column read the row's last quad.
  const char *fb = reinterpret_cast<const char *>(a.f);
  const int64_t szb = g.sz * 4;
  const int cl = min(c0, (mx - 1) & ~3);
  const uint32_t xoff = (uint32_t)(cl * SX * 4);
  uint32_t roff[NR];  // byte offsets of rows y0-1 .. y0+R (wave-uniform)
#pragma unroll
  for (int i = 0; i < NR; i++)
    roff[i] = (uint32_t)((int64_t)min(max(y0 - 1 + i, 0), my - 1) * g.sy * 4);
  uint32_t hoff;
  {
    int hi, col;
    if (lane < 16) {
      hi = lane;
      col = max(x0 - 1, 0);
    } else if (lane < 48) {
      hi = lane < 32 ? lane - 16 : 0;
      col = x0;
    } else {
      hi = lane - 48;
      col = min(x0 + kQuadCols, mx - 1);
    }
    hi = min(hi, NR - 1);
    hoff = (uint32_t)(((int64_t)min(max(y0 - 1 + hi, 0), my - 1) * g.sy + (int64_t)col * SX) * 4);
  }
  auto plane_rsrc = [&](int z) {
    const int64_t pz = (int64_t)min(max(z, 0), mz - 1) * szb;
    const int64_t rem = a.fbytes - pz;
    return rsrc_n(fb + pz, rem > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)rem);
  };
  auto load = [&](int z, QPlane<R, SX> &d) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(z);
#pragma unroll
    for (int i = 0; i < NR; i++) {
      d.raw[0][i] = ld128(r, xoff, roff[i]);
      if (SX == 2) d.raw[SX - 1][i] = ld128(r, xoff + 16, roff[i]);
    }
    d.h = ld_f32(r, hoff);
  };
  // x+1 neighbour of each row's last column: the next lane's first column,
  // at lane 63 the right halo
  auto derive_s = [&](const QPlane<R, SX> &d, float *s) {
    static_for<NR - 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value + 1;  // row 0 needs none
      const float go = mov_dpp_f<0x110 + (15 - i)>(d.h);  // row_shr: lane 63 <- lane 48+i
      s[i] = dpp_f<kDppShl1>(go, d.v(i).x);
    });
  };
  // column x0 of every row, lane i <- lane 16+i (rows 0 and 1 of the
  // wave swapped)
  auto derive_a = [&](const QPlane<R, SX> &d) {
    const unsigned hb = __float_as_uint(d.h);
    return __uint_as_float(__builtin_amdgcn_permlane16_swap(hb, hb, false, false)[1]);
  };
  // P bits (1,0,0), (1,1,0), (1,0,1), (1,1,1) of column x0-1 of row i, in
  // byte 3 of lane i (the byte the x-shift moves into lane 0)
  auto halo_p = [&](float hz, float az, float az1) {
    const float azu = mov_dpp_f<0x101>(az);  // row_shl:1 -- the row above
    const float az1u = mov_dpp_f<0x101>(az1);
    unsigned m = push_sign(0u, az1u - hz);
    m = push_sign(m, az1 - hz);
    m = push_sign(m, azu - hz);
    m = push_sign(m, az - hz);
    return m << 24;
  };
  // P bytes of a row C (x+1 of its last column sC), with the row above Uq,
  // the plane above Bq and the row above that BUq.  Pushed from column 3
  // down to 0 and direction 6 down to 0; the push of direction 0 of columns
  // 3..1 takes one more bit, the unused bit 7 of the next byte.
  auto prow = [&](const float4 &C, float sC, const float4 &Uq, float sU, const float4 &Bq,
                  float sB, const float4 &BUq, float sBU) {
    const float c[4] = {C.x, C.y, C.z, C.w}, xc[4] = {C.y, C.z, C.w, sC};
    const float u[4] = {Uq.x, Uq.y, Uq.z, Uq.w}, xu[4] = {Uq.y, Uq.z, Uq.w, sU};
    const float b[4] = {Bq.x, Bq.y, Bq.z, Bq.w}, xb[4] = {Bq.y, Bq.z, Bq.w, sB};
    const float bu[4] = {BUq.x, BUq.y, BUq.z, BUq.w}, xbu[4] = {BUq.y, BUq.z, BUq.w, sBU};
    unsigned m = 0;
    static_for<4>([&](auto ec) {
      constexpr int e = 3 - decltype(ec)::value;
      m = push_sign(m, bu[e] - c[e]);   // 6 (0,1,1)
      m = push_sign(m, b[e] - c[e]);    // 5 (0,0,1)
      m = push_sign(m, u[e] - c[e]);    // 4 (0,1,0)
      m = push_sign(m, xbu[e] - c[e]);  // 3 (1,1,1)
      m = push_sign(m, xb[e] - c[e]);   // 2 (1,0,1)
      m = push_sign(m, xu[e] - c[e]);   // 1 (1,1,0)
      m = push_bits(m, xc[e] - c[e], e > 0 ? 30 : 31);  // 0 (1,0,0)
    });
    return m;
  };
  // The row below the tile: only its bits 1, 3, 4, 6 are read (the
  // directions with dy = 1); the pushes skip the others.
  auto prow0 = [&](const float4 &C, const float4 &Uq, float sU, const float4 &BUq, float sBU) {
    const float c[4] = {C.x, C.y, C.z, C.w};
    const float u[4] = {Uq.x, Uq.y, Uq.z, Uq.w}, xu[4] = {Uq.y, Uq.z, Uq.w, sU};
    const float bu[4] = {BUq.x, BUq.y, BUq.z, BUq.w}, xbu[4] = {BUq.y, BUq.z, BUq.w, sBU};
    unsigned m = 0;
    static_for<4>([&](auto ec) {
      constexpr int e = 3 - decltype(ec)::value;
      m = push_bits(m, bu[e] - c[e], 30);              // 6, 5
      m = push_bits(m, u[e] - c[e], 31);               // 4
      m = push_bits(m, xbu[e] - c[e], 30);             // 3, 2
      m = push_bits(m, xu[e] - c[e], e > 0 ? 29 : 30);  // 1, 0 (, 7 of the next byte)
    });
    return m;
  };
  // P bytes shifted one column to the right: column x gets column x-1; lane
  // 0 gets the halo bits of column x0-1 (row i's bits in lane i of hp)
  auto pshift = [&](unsigned p, unsigned hpo) {
    return __builtin_amdgcn_alignbyte(p, dpp_u<kDppShr1>(hpo, p), 3);
  };

  // x-boundary vertices: masks (0xFF in the lane and column that holds
  // column 0 / column mx-1 of the level, else 0) that select their codes
  // from the x-boundary tables; at full resolution mx-1 is always column 3
  // of its lane (mx is a multiple of 4)
  const uint8_t *const txl = slut + kQuadTableSize;         // x-low boundary codes
  const uint8_t *const txh = slut + kQuadTableSize + 1024;  // x-high boundary codes
  const unsigned mxl = c0 == 0 ? 0xFFu : 0u;
  unsigned mxh[4];
#pragma unroll
  for (int e = 0; e < 4; e++) mxh[e] = c0 + e == mx - 1 ? 0xFFu : 0u;
  // code stores: lane offsets, past the record limit for columns past the
  // level (the hardware drops those stores), and no stores at all without a
  // codes array
  uint32_t cvo[SX == 1 ? 1 : 4];
  if (SX == 1) {
    cvo[0] = nval == 4 ? (uint32_t)c0 : 0x80000000u;
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) cvo[e] = e < nval ? (uint32_t)(c0 + e) * SX : 0x80000000u;
  }
  const uint32_t crec = a.codes ? (uint32_t)g.sz : 0u;  // bytes of a plane of codes

  QPlane<R, SX> F[NS];
  float S[NS][NR];
  float AV[NS];
  unsigned PB[2][R + 1], PSB[2][R + 1];
  uint64_t special = 0;  // lanes with a special centre (wave-uniform)

  // Prologue: planes z0-1, z0 and z0+1; P of plane z0-1.
  load(z0 - 1, F[0]);
  load(z0, F[1]);
  static_for<NS - 2>([&](auto kc) {
    constexpr int k = decltype(kc)::value + 2;
    load(min(z0 + k - 1, zlim), F[k]);
  });
  derive_s(F[0], S[0]);
  AV[0] = derive_a(F[0]);
  derive_s(F[1], S[1]);
  AV[1] = derive_a(F[1]);
  {
    const unsigned hp = halo_p(F[0].h, AV[0], AV[1]);
    PB[0][0] = prow0(F[0].v(0), F[0].v(1), S[0][1], F[1].v(1), S[1][1]);
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value + 1;
      PB[0][i] = prow(F[0].v(i), S[0][i], F[0].v(i + 1), S[0][i + 1], F[1].v(i), S[1][i],
                      F[1].v(i + 1), S[1][i + 1]);
    });
    static_for<R + 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      PSB[0][i] = pshift(PB[0][i], i == 0 ? hp : mov_dpp_u<0x100 + (i > 0 ? i : 1)>(hp));
    });
  }

  // Bitmask words: lane 16 k + 15 ends with word 4 tx + k of each row; one
  // store per step writes the R rows' words, row j from lane 16 k + 15 - j.
  // Every lane takes part in it: the other lanes' offsets lie past the
  // record limit, so the hardware drops their writes, and the store needs no
  // branch (a branch around a store makes the compiler wait for the stores
  // of one step before the next step's loads may be used).
  const int wshift = 4 * (lane & 7);
  const uint32_t wrec = (uint32_t)g.rowwords * 8u;  // bytes of a row of words
  const int wrow = 15 - (lane & 15);
  const uint32_t wvo = wrow < R && 4 * tp.tx + (lane >> 4) < g.rowwords
                           ? (uint32_t)(4 * tp.tx + (lane >> 4)) * 8u + (uint32_t)wrow * wrec
                           : 0x80000000u;
  const unsigned vnib = (1u << nval) - 1u;  // valid columns of this lane
  const uint32_t sy = (uint32_t)g.sy;
  uint8_t *const codes = a.codes;

  auto step = [&](auto uc, int z) {
    constexpr int u = decltype(uc)::value;
    // slots of planes z, z+1 and z+NS-1 (the slot plane z-1 frees)
    constexpr int s0 = (u + 1) % NS, s1 = (u + 2) % NS, s2 = u % NS;
    constexpr int pc = (u + 1) % 2, pp = u % 2;                    // P of planes z, z-1
    F[s2].keep();
    load(min(z + NS - 1, zlim), F[s2]);
    derive_s(F[s1], S[s1]);
    AV[s1] = derive_a(F[s1]);
    const unsigned hp = halo_p(F[s0].h, AV[s0], AV[s1]);
    PB[pc][0] = prow0(F[s0].v(0), F[s0].v(1), S[s0][1], F[s1].v(1), S[s1][1]);
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value + 1;
      PB[pc][i] = prow(F[s0].v(i), S[s0][i], F[s0].v(i + 1), S[s0][i + 1], F[s1].v(i),
                       S[s1][i], F[s1].v(i + 1), S[s1][i + 1]);
    });
    static_for<R + 1>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      PSB[pc][i] = pshift(PB[pc][i], i == 0 ? hp : mov_dpp_u<0x100 + (i > 0 ? i : 1)>(hp));
    });
    const unsigned az = GEN ? (z == 0 ? QAZM : 0u) | (z == mz - 1 ? QAZP : 0u) : 0u;
    const __amdgpu_buffer_rsrc_t crs = rsrc_n(codes + (int64_t)z * g.sz, crec);
    uint32_t wq[R][2];  // each row's bitmask word (low, high half)
    static_for<R>([&](auto ic) {
      constexpr int i = decltype(ic)::value + 1;
      const int y = y0 + i - 1;
      const unsigned P = PB[pc][i];
      const unsigned N = (PSB[pc][i] & 0x01010101u) | (PSB[pc][i - 1] & 0x02020202u) |
                         (PSB[pp][i] & 0x04040404u) | (PSB[pp][i - 1] & 0x08080808u) |
                         (PB[pc][i - 1] & 0x10101010u) | (PB[pp][i] & 0x20202020u) |
                         (PB[pp][i - 1] & 0x40404040u);
      unsigned idx[4], code[4];
      static_for<4>([&](auto ec) {
        constexpr unsigned e = decltype(ec)::value;
        idx[e] = __builtin_amdgcn_perm(N, P, 0x0C0C0000u | ((4u + e) << 8) | e);
        code[e] = slut[idx[e]];
      });
      const float4 C = F[s0].v(i);
      special |= wave_ballot(special_centre(C.x) | special_centre(C.y) |
                             special_centre(C.z) | special_centre(C.w));
      bool cr[4];  // critical
      const unsigned ayz = GEN ? az | (y == 0 ? QAYM : 0u) | (y == my - 1 ? QAYP : 0u) : 0u;
      if (GEN && ayz != 0u) {
        // a boundary row or plane: every vertex of the row
        static_for<4>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          const unsigned A = ayz | (c0 + e == 0 ? QAXM : 0u) | (c0 + e == mx - 1 ? QAXP : 0u);
          code[e] = quad_boundary(slut, idx[e], A);
          cr[e] = (code[e] & 0xBFu) != 0x09u;
        });
      } else {
        // x-boundary columns: codes from the x-boundary tables, indexed
        // without the absent bits, computed in every lane and kept where the
        // mask selects them (no branch)
        const unsigned cl = txl[__builtin_amdgcn_ubfe(idx[0], 0, 7) |
                                (__builtin_amdgcn_ubfe(idx[0], 12, 3) << 7)];
        code[0] = (cl & mxl) | (code[0] & ~mxl);
        static_for<4>([&](auto ec) {
          constexpr int e = decltype(ec)::value;
          if (SX == 2 || e == 3) {
            const unsigned ch = txh[__builtin_amdgcn_ubfe(idx[e], 4, 3) |
                                    (__builtin_amdgcn_ubfe(idx[e], 8, 7) << 3)];
            code[e] = (ch & mxh[e]) | (code[e] & ~mxh[e]);
          }
          const bool edge = SX == 2 || e == 0 || e == 3;
          cr[e] = edge ? (code[e] & 0xBFu) != 0x09u : code[e] != 0x09u;
        });
      }
      {
        // a row past the level (odd my) stores nothing: its offsets lie
        // past the record limit, with no branch around the store
        const bool rv = !GEN || y < my;
        if (SX == 1) {
          const unsigned packed = code[0] | (code[1] << 8) | (code[2] << 16) | (code[3] << 24);
          __builtin_amdgcn_raw_buffer_store_b32(packed, crs, rv ? cvo[0] : 0x80000000u,
                                                (uint32_t)y * sy, 0);
        } else if (CODES) {
#pragma unroll
          for (int e = 0; e < 4; e++)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)code[e], crs,
                                                 rv ? cvo[e] : 0x80000000u, (uint32_t)y * sy, 0);
        }
        // this lane's four bits, moved to their place in its half of the
        // word of its sixteen-lane row; three DPP ORs gather lanes 0..7 of
        // the row (the low half) in lane 7 and lanes 8..15 (the high half)
        // in lane 15, and one more brings the low half to lane 15
        unsigned nib = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) nib |= (unsigned)cr[e] << e;
        if (!full) nib &= vnib;
        uint32_t wv = nib << wshift;
        static_for<3>([&](auto dc) {
          constexpr int d = 1 << decltype(dc)::value;
          wv |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wv, 0x110 + d, 0xF, 0xF, true);
        });
        const uint32_t wlo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wv, 0x118, 0xF, 0xF, true);
        wq[i - 1][0] = wlo;
        wq[i - 1][1] = wv;
      }
    });
    // row j's word moves from lane 16 k + 15 to lane 16 k + 15 - j; rows
    // past the level lie past the record limit
    uint32_t dlo = wq[0][0], dhi = wq[0][1];
    static_for<R - 1>([&](auto jc) {
      constexpr int j = decltype(jc)::value + 1;
      const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wq[j][0], 0x100 + j, 0xF, 0xF, true);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wq[j][1], 0x100 + j, 0xF, 0xF, true);
      dlo = wrow == j ? lo : dlo;
      dhi = wrow == j ? hi : dhi;
    });
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 wd = {dlo, dhi};
    const uint32_t nrow = GEN ? (uint32_t)min(R, my - y0) : (uint32_t)R;
    __builtin_amdgcn_raw_buffer_store_b64(
        wd, rsrc_n(g.bits + ((int64_t)z * my + y0) * g.rowwords, nrow * wrec), wvo, 0, 0);
  };

  // the prologue's loads have landed: each step's wait then counts only the
  // previous step's loads and lets its stores run on
  __builtin_amdgcn_s_waitcnt(kWaitVmem);
  for (int zb = z0; zb < z1; zb += U) {
    static_for<U>([&](auto uc) {
      const int z = zb + decltype(uc)::value;
      if (z < z1) step(uc, z);
    });
  }

  // Rare: centres whose differences may not carry the order.  Their codes
  // and bits are redone by comparisons (the others are exact: a difference
  // with one finite non-zero end has the right sign).
  if (special) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this wave's stores first
    auto fetch = [&](int x, int y, int z) {
      x = min(max(x, 0), mx - 1);
      y = min(max(y, 0), my - 1);
      z = min(max(z, 0), mz - 1);
      return a.f[(int64_t)x * SX + (int64_t)y * g.sy + (int64_t)z * g.sz];
    };
#pragma unroll 1
    for (int z = z0; z < z1; z++) {
#pragma unroll 1
      for (int r = 0; r < R && y0 + r < my; r++) {
        const int y = y0 + r;
#pragma unroll 1
        for (int e = 0; e < 4; e++) {
          const int x = c0 + e;
          const float c = x < mx ? fetch(x, y, z) : 1.0f;
          const bool sp = x < mx && special_centre(c);
          if (!wave_ballot(sp)) continue;
          if (sp) {
            nan_seen |= c != c;
            unsigned p = 0, n = 0;
#pragma unroll 1
            for (int j = 0; j < 7; j++) {
              const float vp = fetch(x + kQD[j][0], y + kQD[j][1], z + kQD[j][2]);
              const float vn = fetch(x - kQD[j][0], y - kQD[j][1], z - kQD[j][2]);
              p |= (unsigned)(vp < c) << j;
              n |= (unsigned)(c < vn) << j;
            }
            const unsigned idx = p | (n << 8);
            const unsigned A = (x == 0 ? QAXM : 0u) | (x == mx - 1 ? QAXP : 0u) |
                               (y == 0 ? QAYM : 0u) | (y == my - 1 ? QAYP : 0u) |
                               (z == 0 ? QAZM : 0u) | (z == mz - 1 ? QAZP : 0u);
            const unsigned code = A ? quad_boundary(slut, idx, A) : (unsigned)slut[idx];
            if (codes) codes[(int64_t)z * g.sz + (int64_t)y * g.sy + (int64_t)x * SX] = (uint8_t)code;
            unsigned long long *w = reinterpret_cast<unsigned long long *>(
                g.bits + ((int64_t)z * my + y) * g.rowwords + (x >> 6));
            const unsigned long long bit = 1ull << (x & 63);
            if ((code & 0xBFu) != 0x09u)
              atomicOr(w, bit);
            else
              atomicAnd(w, ~bit);
          }
        }
      }
    }
  }
}

// LISTED: tiles from the region-ordered per-XCD lists (QuadArgs::tile_list)
// instead of a grid-stride walk over the level.
template <int R, int SX, bool LISTED, bool CODES>
__global__ __launch_bounds__(64 * kQuadBlockWaves)
__attribute__((amdgpu_waves_per_eu(kQuadWavesPerSimd)))
void classify3d_quad_kernel(QuadArgs a) {
  constexpr int NW = kQuadBlockWaves;
  __shared__ __attribute__((aligned(16))) uint8_t slut[kQuadTableBytes];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  {
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(a.lut);
    uint4 *s = reinterpret_cast<uint4 *>(slut);
    for (int i = tid; i < kQuadTableBytes / 16; i += 64 * NW) s[i] = gsrc[i];
  }
  __syncthreads();
  bool nan_seen = false;
  // Tiles: grid-stride over the level, or (region order) this XCD's list,
  // one tile per increment of its counter.
  const int x = (int)blockIdx.x % kXcds;
  const int beg = LISTED ? a.xcd_off[x] : 0, nlist = LISTED ? a.xcd_off[x + 1] - beg : 0;
  const int nwaves = (int)gridDim.x * NW;
  int t0 = xcd_block_id() * NW + w;
  for (;;) {
    int t;
    if (LISTED) {
      int i = 0;
      if (lane == 0) i = atomicAdd(&a.queue[kCounterStride * x], 1);
      i = __builtin_amdgcn_readfirstlane(i);
      if (i >= nlist) break;
      t = a.tile_list[beg + i];
    } else {
      if (t0 >= a.lv.ntiles) break;
      t = t0;
      t0 += nwaves;
    }
    const TilePos p = tile_pos(a.lv, t);
    const int y0 = p.ty * R, z0 = p.zc * a.lv.zchunk;
    const bool inner = y0 >= 1 && y0 + R <= a.lv.my - 1 && z0 >= 1 &&
                       z0 + a.lv.zchunk <= a.lv.mz - 1;
    if (inner)
      quad_tile<R, SX, false, CODES>(a, t, lane, slut, nan_seen);
    else
      quad_tile<R, SX, true, CODES>(a, t, lane, slut, nan_seen);
    if (LISTED) {
      // the region's last tile stamps the clock once this tile's stores
      // have completed (a wait on the vector memory counter only: a
      // release fence at device scope would also write back the XCD's L2)
      __builtin_amdgcn_s_waitcnt(kWaitVmem);
      if (lane == 0) {
        const int r = ((p.zc * a.lv.zchunk * SX) / a.region_edge) * a.nry +
                      (p.ty * R * SX) / a.region_edge;
        if (atomicSub(&a.region_left[kCounterStride * r], 1u) == 1u)
          a.region_stamp[r] = __builtin_amdgcn_s_memrealtime();
      }
    }
  }
  if (wave_ballot(nan_seen) && lane == 0) *a.nan_flag = a.gen;
}

// Quad tiles per wave of a launch (the kernel strides over tiles by the
// grid's wave count).
#ifndef PCRIT_QUAD_TILE_ROUNDS
#define PCRIT_QUAD_TILE_ROUNDS 2
#endif
constexpr int kQuadTileRounds = PCRIT_QUAD_TILE_ROUNDS;
// Tile depth: the deepest multiple of 2 up to kQuadZChunk that still gives
// kQuadWantTiles tiles.
constexpr int64_t kQuadWantTiles = 4096;

}  // namespace

void plan_level_quad(LevelDesc &l, int zmax) {
  l.ntx = (l.mx + kQuadCols - 1) / kQuadCols;
  l.nty = (l.my + kQuadRows - 1) / kQuadRows;
  int d = kQuadZChunk;
  while (d > 2 && (int64_t)l.ntx * l.nty * ((l.mz + d - 1) / d) < kQuadWantTiles) d -= 2;
  if (zmax > 0) {
    int p = 2;
    while (2 * p <= std::min(d, zmax)) p *= 2;
    d = p;
  }
  l.zchunk = d;
  l.ntiles = l.ntx * l.nty * ((l.mz + l.zchunk - 1) / l.zchunk);
  fast_divisor((uint32_t)l.ntx, &l.ntx_mul, &l.ntx_shift);
  fast_divisor((uint32_t)l.nty, &l.nty_mul, &l.nty_shift);
}

bool quad_eligible(const float *field, int64_t nx, int64_t s, int dim) {
  // 16-byte loads of four (stride 1) or eight (stride 2) samples need rows
  // that start on 16-byte boundaries
  return dim == 3 && (s == 1 || s == 2) && ((uintptr_t)field & 15u) == 0 &&
         (nx * s) % 4 == 0;
}

hipError_t launch_classify_quad(const QuadArgs &a, hipStream_t st) {
  const int64_t per_block = (int64_t)kQuadBlockWaves * kQuadTileRounds;
  int g = (int)((a.lv.ntiles + per_block - 1) / per_block);
  // region order: every XCD drains its own list, so each needs workgroups
  // (a multiple of kXcds); beyond what the chip holds at once more add
  // nothing
  if (a.tile_list) g = std::min((g + kXcds - 1) / kXcds * kXcds, 2048);
  const dim3 grid((unsigned)(g > 0 ? g : 1)), block(64 * kQuadBlockWaves);
  if (a.lv.sx != 1 && a.lv.sx != 2) return hipErrorInvalidValue;
  const bool codes = a.codes != nullptr;
  if (a.tile_list) {
    if (a.lv.sx == 1)
      hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 1, true, true>), grid, block, 0, st, a);
    else if (codes)
      hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 2, true, true>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 2, true, false>), grid, block, 0, st, a);
  } else if (a.lv.sx == 1) {
    hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 1, false, true>), grid, block, 0, st, a);
  } else if (codes) {
    hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 2, false, true>), grid, block, 0, st, a);
  } else {
    hipLaunchKernelGGL((classify3d_quad_kernel<kQuadRows, 2, false, false>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace pcrit
