// Internal declarations of the pcrit GPU library (host driver + kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcrit {

constexpr int kLut3Size = 1 << 14;
constexpr int kLut2Size = 1 << 6;

// Neighbour offsets (dx, dy, dz) of the 3D grid triangulation; bit j of a
// polarity mask refers to kOff3[j].  Grouped by plane so that the kernels
// can fetch them plane by plane.
constexpr int kOff3[14][3] = {
    {0, 0, -1}, {-1, 0, -1}, {0, -1, -1}, {-1, -1, -1},              // dz = -1
    {-1, 0, 0}, {1, 0, 0},   {0, -1, 0},  {0, 1, 0}, {-1, -1, 0}, {1, 1, 0},
    {0, 0, 1},  {1, 0, 1},   {0, 1, 1},   {1, 1, 1}};                // dz = +1
// 2D neighbour offsets (dx, dy).
constexpr int kOff2[6][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, 1}};

// Bits of the neighbours that lie on a given side: axis a (0 = x, 1 = y,
// 2 = z), side -1 or +1.  Used to build the absent-neighbour mask of a
// boundary vertex.
constexpr unsigned side_mask3(int axis, int side) {
  unsigned m = 0;
  for (int j = 0; j < 14; j++)
    if (kOff3[j][axis] == side) m |= 1u << j;
  return m;
}
constexpr unsigned side_mask2(int axis, int side) {
  unsigned m = 0;
  for (int j = 0; j < 6; j++)
    if (kOff2[j][axis] == side) m |= 1u << j;
  return m;
}

// Host: link-pattern tables (see pcrit_link_table in pcrit.h).
void build_link_table3(uint8_t *table);
void build_link_table2(uint8_t *table);

// Look-back chunk of the compaction kernel: 256 threads x 4 words of 64 bits.
constexpr int kCompactThreads = 256;
constexpr int kCompactWordsPerThread = 4;
constexpr int kChunkWords = kCompactThreads * kCompactWordsPerThread;

struct ClassifyArgs {
  const float *f;       // full-resolution field
  uint8_t *codes;       // full-resolution code bytes
  uint64_t *bits;       // critical bitmask of this level, one padded row of
                        // rowwords words per (y, z) level row
  const uint8_t *lut;   // link-pattern table (device)
  int64_t sx, sy, sz;   // element strides of one level step along x, y, z
  int mx, my, mz;       // level sizes (mz = 1 in 2D)
  int rowwords;         // ceil(mx / 64)
  int zchunk;           // planes (3D) / rows (2D) per block
  int ntx, nty;         // tiles along x and y (3D) / x (2D)
  // progressive refinement (level k < k_max)
  const uint64_t *prev_bits;  // critical bitmask of level k+1
  int prev_rowwords, prev_my;
  unsigned *reclass;          // counter of re-classified old vertices
  // error reporting: flags hold the generation number of the failing call
  unsigned *nan_flag;
  unsigned gen;
  // reset of the look-back state used by the compaction that follows
  uint64_t *lb_state;
  int lb_n;
  unsigned *lb_counter;
};

struct CompactArgs {
  const uint64_t *bits;
  int64_t words;        // rows * rowwords
  int rowwords;
  int my;               // level rows per plane (rows of a 2D level)
  int64_t s;            // level stride
  int64_t nx, ny;       // full-resolution sizes
  uint32_t *crit;
  uint8_t *crit_codes;  // may be null
  const uint8_t *codes;
  int64_t cap;
  int64_t *level_base;  // reads level_base[slot], writes level_base[slot+1]
  int slot;
  int64_t *count_dev;   // may be null
  unsigned *nan_flag;
  unsigned *err_flag;
  unsigned gen;
  uint64_t *lb_state;
  unsigned *lb_counter;
  int nchunks;
  unsigned *zero_next;  // counter to clear for the next level (may be null)
};

hipError_t launch_classify3d(const ClassifyArgs &a, bool progressive,
                             hipStream_t st);
hipError_t launch_classify2d(const ClassifyArgs &a, bool progressive,
                             hipStream_t st);
hipError_t launch_compact(const CompactArgs &a, hipStream_t st);

// Launch geometry helpers (host).
int classify3d_zchunk(int mx, int my, int mz);
int classify2d_ychunk(int mx, int my);
constexpr int kTile3X = 64;
constexpr int kTile3Y = 4;
constexpr int kTile2X = 256;

}  // namespace pcrit
