// Device helpers shared by the classification kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "pcrit_internal.h"

namespace pcrit {
namespace dev {

// Hardware hands consecutive workgroups to the 8 XCDs round-robin; renumber
// them so that each XCD (and its L2) gets a contiguous run of tiles, whose
// halo rows it then shares.
__device__ __forceinline__ int xcd_block_id() {
  const int G = gridDim.x, b = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = b & 7, j = b >> 3;
  return xcd * q + min(xcd, r) + j;
}

// Orders this wave's LDS reads after its earlier LDS writes by other lanes
// (a wave executes its LDS instructions in order; this only stops the
// compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kDppShl1 = 0x130;  // wave_shl:1 -- lane i reads lane i+1
constexpr int kDppShr1 = 0x138;  // wave_shr:1 -- lane i reads lane i-1

// x-1 / x+1 neighbour across lanes: lane i reads lane i-1 (i+1); lane 0
// (63) keeps `halo`, which holds the sample left (right) of the tile.
__device__ __forceinline__ float shift_left(float halo, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(
      __float_as_int(halo), __float_as_int(v), kDppShr1, 0xF, 0xF, false));
}
__device__ __forceinline__ float shift_right(float halo, float v) {
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
__device__ __forceinline__ uint64_t wave_ballot(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}
// this lane's bit of a wave mask
__device__ __forceinline__ bool lane_bit(uint64_t m) {
  return __builtin_amdgcn_inverse_ballot_w64(m);
}

// Buffer resources: a scalar base address and a 32-bit lane offset per
// access, so address arithmetic stays off the vector ALU.  (Raw buffer,
// no swizzle; the record limit is the full 32-bit offset range.)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1,
                                           0x00020000);
}
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ unsigned ld_u16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
}
__device__ __forceinline__ unsigned ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}
__device__ __forceinline__ void st_u8(__amdgpu_buffer_rsrc_t r, uint32_t off, unsigned v) {
  __builtin_amdgcn_raw_buffer_store_b8((unsigned char)v, r, off, 0, 0);
}
__device__ __forceinline__ void st_u16(__amdgpu_buffer_rsrc_t r, uint32_t off, unsigned v) {
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, off, 0, 0);
}

// floor(n / d) for 0 <= n < 2^31 from the divisor's multiplier and shift
__device__ __forceinline__ int fdiv(int n, uint32_t mul, int shift) {
  return (int)(((uint64_t)(uint32_t)n * mul) >> shift);
}
// tile index -> (tile column, tile row, chunk) of a level
struct TilePos {
  int tx, ty, zc;
};
__device__ __forceinline__ TilePos tile_pos(const LevelDesc &g, int t) {
  const int rest = fdiv(t, g.ntx_mul, g.ntx_shift);
  const int zc = fdiv(rest, g.nty_mul, g.nty_shift);
  return {t - rest * g.ntx, rest - zc * g.nty, zc};
}

// Calls f(std::integral_constant<int, 0>{}) .. f(<N-1>{}).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace dev
}  // namespace pcrit
