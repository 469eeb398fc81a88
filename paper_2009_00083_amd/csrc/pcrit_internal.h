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

// Compaction chunk: 256 threads x 4 words of 64 bits (65536 vertices).
constexpr int kCompactThreads = 256;
constexpr int kCompactWordsPerThread = 4;
constexpr int kChunkWords = kCompactThreads * kCompactWordsPerThread;

// Tiles of the classification kernels.  Every wave owns a tile of 64
// consecutive x (one sample per lane) by kTile3Y rows (3D) or one row (2D)
// and marches it along the slowest axis; the waves of a block only share
// the link-pattern table.
constexpr int kWavesPerBlock = 4;
constexpr int kTile3Y = 2;    // rows per 3D wave tile
constexpr int kZChunk3 = 24;  // planes per 3D wave tile
constexpr int kYChunk2 = 60;  // rows per 2D wave tile

struct ClassifyArgs {
  const float *f;       // full-resolution field
  uint8_t *codes;       // full-resolution code bytes
  uint64_t *bits;       // critical bitmask of this level, one padded row of
                        // rowwords words per (y, z) level row
  const uint8_t *lut;   // link-pattern table (device)
  int64_t sx, sy, sz;   // element strides of one level step along x, y, z
  int mx, my, mz;       // level sizes (mz = 1 in 2D)
  int rowwords;         // ceil(mx / 64)
  int zchunk;           // planes (3D) / rows (2D) per wave tile, a multiple
                        // of 6, at most kZChunk3 / kYChunk2
  int ntx, nty, nzc;    // wave tiles along x, y, z (2D: x, 1, y)
  int ntiles;
  // progressive refinement: polarity masks of the previous (coarser) level,
  // dense in its level-local index order (uint16 in 3D, uint8 in 2D), and
  // the masks of this level for the next one (same layout, may be null)
  const void *prev_masks;
  int pmx, pmy;         // sizes of the previous level along x and y
  void *masks;
  unsigned *reclass_part;  // progressive: one count per block
  unsigned *nan_flag;      // set to gen if a level sample is NaN
  unsigned gen;
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
  unsigned gen;
  int *counts;          // per-chunk critical counts
  int nchunks;
  const unsigned *reclass_part;  // summed into *reclass_out (may be null)
  int reclass_n;
  unsigned *reclass_out;
};

// The classification launchers store the number of blocks they launched
// (entries of reclass_part written) in *grid_out.
hipError_t launch_classify3d(ClassifyArgs a, bool read_prev, bool write_masks,
                             hipStream_t st, int *grid_out);
hipError_t launch_classify2d(ClassifyArgs a, bool read_prev, bool write_masks,
                             hipStream_t st, int *grid_out);
hipError_t launch_compact(const CompactArgs &a, hipStream_t st);

// Number of persistent blocks a classification launch uses (the size of
// the per-block reclass array).
int classify_max_blocks();

}  // namespace pcrit
