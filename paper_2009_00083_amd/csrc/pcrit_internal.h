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

// Quad tiles (full-resolution and stride-2 levels of 3D grids, four
// columns per lane).  Their table index is built from edge signs: the seven
// neighbour offsets with all components >= 0 ("positive" directions, the
// later neighbours in index order) in this order,
constexpr int kQD[7][3] = {{1, 0, 0}, {1, 1, 0}, {1, 0, 1}, {1, 1, 1},
                           {0, 1, 0}, {0, 0, 1}, {0, 1, 1}};
// bit j (0..6): sign bit of f(v + d_j) - f(v), i.e. 1 iff that neighbour
// comes before v; bit 8 + j: sign bit of f(v) - f(v - d_j), i.e. 1 iff
// v - d_j comes after v; bit 7 carries no information and bit 15 is 0.
constexpr int kQuadTableSize = 1 << 15;
// Followed by the codes of x-boundary vertices (two tables of 1024 bytes):
// column 0 indexed by bits 0-6 and 12-14 of the index (the others are the
// absent neighbours), column mx-1 by bits 4-6 and 8-14.
constexpr int kQuadTableBytes = kQuadTableSize + 2048;
constexpr unsigned kQPos = 0x007Fu, kQNeg = 0x7F00u;
// Absent-neighbour bits of a vertex on the low (side -1) or high (+1) end
// of axis a (0 = x, 1 = y, 2 = z) in that index.
constexpr unsigned quad_side(int axis, int side) {
  unsigned m = 0;
  for (int j = 0; j < 7; j++)
    if (kQD[j][axis] == 1) m |= side < 0 ? 1u << (8 + j) : 1u << j;
  return m;
}
// The quad table from the link-pattern table: entry of index i = entry of
// the polarity mask i describes.
void build_quad_table3(const uint8_t *table3, uint8_t *quad);  // kQuadTableBytes

// Compaction chunk: 256 threads x 4 words of 64 bits (65536 vertices).
constexpr int kCompactThreads = 256;
constexpr int kCompactWordsPerThread = 4;
constexpr int kChunkWords = kCompactThreads * kCompactWordsPerThread;

// Tiles of the classification kernels.  A wave holds 64 consecutive
// columns (one per lane) of kTile3Y rows (3D) or one row (2D), plus the
// columns left and right of the tile from a halo load, and marches them along
// the slowest axis; the waves of a block only share the link-pattern table.
// A critical-bitmask word covers the kTileCols columns of one tile row: bit
// L is column word*kTileCols + L.
constexpr int kTileCols = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kTile3Y = 2;    // rows per 3D wave tile
constexpr int kZChunk3 = 24;  // planes per 3D wave tile
// Launches that store masks stage twice as many bytes per vertex in LDS;
// their tiles are shallower so that five blocks fit on a CU.
constexpr int kZChunk3Masks = 8;
constexpr int zchunk_cap3(bool write_masks) { return write_masks ? kZChunk3Masks : kZChunk3; }
constexpr int kYChunk2 = 60;  // rows per 2D wave tile
constexpr int kUnroll3 = 4;   // 3D march unroll (ring of planes in registers)
constexpr int kUnroll2 = 12;  // 2D march unroll (rows in registers)

// Polarity bits of the offsets with a larger linear index (first non-zero
// of (dz, dy, dx) positive).  The kernels build a raw mask whose bit j is
// the sign bit of the difference taken towards the larger index; the true
// polarity mask is raw ^ kPos.  The device table is stored permuted so that
// it is indexed by the raw mask directly.
constexpr unsigned kPos3 = 0x3EA0u;
constexpr unsigned kPos2 = 0x2Au;

// Levels of at most kSmallLevel vertices are launch-latency bound; the
// progressive driver classifies and compacts all of them in one launch each
// (up to kMaxFused levels).
constexpr int64_t kSmallLevel = 1 << 22;
constexpr int kMaxFused = 16;

// One level as the classification kernels see it.
struct LevelDesc {
  const float *f;         // full-resolution field of this level
  uint8_t *codes;         // its full-resolution code bytes
  int64_t sx, sy, sz;     // element strides of one level step along x, y, z
  int mx, my, mz;         // level sizes (mz = 1 in 2D)
  int rowwords;           // ceil(mx / 64)
  int zchunk;             // planes (3D) / rows (2D) per wave tile
  int ntx, nty, ntiles;   // wave tiles along x and y (3D); x (2D); total
  // n / ntx and n / nty for 0 <= n < 2^31 as (n * mul) >> shift
  uint32_t ntx_mul, nty_mul;
  int ntx_shift, nty_shift;
  int tile_begin;         // first tile of this level in a fused launch
  uint64_t *bits;         // critical bitmask, rowwords words per level row
  uint8_t *lcodes;        // dense level-local codes (fused levels) or null
  const void *prev_masks; // previous level's polarity masks (stored) or null
  int pmx, pmy;           // previous level sizes along x and y
  void *masks;            // this level's polarity masks for the next level
  int write_codes;        // store codes into the full-resolution array
  int dirty;              // test old vertices against the previous level
                          // (its masks from prev_masks if set, else from
                          // the field: the fused launches)
};

struct ClassifyArgs {
  const uint8_t *lut;   // link-pattern table (device)
  int nl;               // levels in this launch (1, or several when fused)
  int ntiles;           // wave tiles of all levels
  LevelDesc lv[kMaxFused];
  unsigned *reclass_acc;   // per level: re-classified old vertices (added to)
  unsigned *nan_flag;      // set to gen if a level sample is NaN
  unsigned gen;
};

// One level as the compaction kernels see it.
struct CompactLevel {
  const uint8_t *codes;   // full-resolution codes of this level's grid
  int64_t nx, ny;         // full-resolution sizes of this level's grid
  const uint64_t *bits;
  int64_t words;        // rows * rowwords
  int rowwords, mx, my;
  int64_t s;            // level stride
  int slot;             // list of this level: level_base[slot] onwards
  int chunk_begin;      // first chunk of this level (chunks in list order)
  const uint8_t *lcodes;  // dense level codes for crit_codes, or null
  unsigned *reclass_out;  // receives reclass_acc[level index], or null
  bool linear;          // full resolution, rows of whole words: index = 64 * word + bit
};

struct CompactArgs {
  int nl;
  int nchunks;          // chunks of all levels
  CompactLevel lv[kMaxFused];
  uint32_t *crit;
  uint8_t *crit_codes;  // may be null
  int64_t cap;
  int64_t *level_base;  // list offsets; [0] is 0
  int64_t *count_dev;   // may be null: total of the last level
  int64_t *publish;     // may be null: level_base[0 .. publish_n) for the
  int publish_n;        // caller (the last one -1 after a NaN sample)
  unsigned *nan_flag;
  unsigned gen;
  int *counts;          // per-chunk critical counts
  unsigned *reclass_acc;  // read into reclass_out, then cleared
};

// Fill the launch geometry of a level (tile depth, tile counts).
void plan_level3(LevelDesc &l, bool write_masks, bool fused);
void plan_level2(LevelDesc &l, bool fused);

// Division by an invariant d in [1, 2^31): with l = ceil(log2 d),
// shift = 31 + l and mul = ceil(2^shift / d) (< 2^32), floor(n / d) equals
// (n * mul) >> shift for every 0 <= n < 2^31.
inline void fast_divisor(uint32_t d, uint32_t *mul, int *shift) {
  int l = 0;
  while ((1ull << l) < d) l++;
  *shift = 31 + l;
  *mul = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
}
// Compaction chunks: kChunkWords words, or kSmallChunkWords for launches of
// at most kSmallLaunchWords words (fused levels, level 1), which would
// otherwise have too few chunks to fill the GPU.  Every chunk sums the
// counts of all chunks before it, so big launches take the big chunks.
constexpr int kSmallWordsPerThread = 1;
constexpr int kSmallChunkWords = kCompactThreads * kSmallWordsPerThread;
constexpr int64_t kSmallLaunchWords = int64_t(1) << 19;
inline bool small_chunks(int64_t launch_words) { return launch_words <= kSmallLaunchWords; }

// Launchers.
// Copies the n list offsets to out (device), the last one -1 if the NaN flag
// holds gen.
hipError_t launch_publish_offsets(const int64_t *level_base, int n,
                                  const unsigned *nan_flag, unsigned gen,
                                  int64_t *out, hipStream_t st);
// fused: several levels or fields in one launch (one tile per wave; old
// vertices tested against masks computed from the field where asked)
hipError_t launch_classify(const ClassifyArgs &a, int dim, bool read_prev,
                           bool write_masks, bool fused, hipStream_t st);
hipError_t launch_compact(const CompactArgs &a, bool small, hipStream_t st);

// Quad tiles: 256 level columns (four per lane, one 16-byte load per row for
// a full-resolution level, two for a stride-2 level) by kQuadRows rows by
// zchunk planes per wave.
constexpr int kQuadCols = 256;
#ifndef PCRIT_QUAD_ROWS
#define PCRIT_QUAD_ROWS 2
#endif
#ifndef PCRIT_QUAD_SLOTS
#define PCRIT_QUAD_SLOTS 3
#endif
#ifndef PCRIT_QUAD_ZCHUNK
#define PCRIT_QUAD_ZCHUNK 16
#endif
constexpr int kQuadRows = PCRIT_QUAD_ROWS;
constexpr int kQuadSlots = PCRIT_QUAD_SLOTS;  // planes held in registers per wave
constexpr int kQuadZChunk = PCRIT_QUAD_ZCHUNK;
#ifndef PCRIT_QUAD_WAVES
#define PCRIT_QUAD_WAVES 3
#endif
// the fewest waves per SIMD the quad kernel is built for: it sets the
// register budget (512 / waves); the full-resolution kernel stays within 128
// registers (four waves) and is scheduled better with the wider budget
constexpr int kQuadWavesPerSimd = PCRIT_QUAD_WAVES;
#ifndef PCRIT_QUAD_BLOCK_WAVES
#define PCRIT_QUAD_BLOCK_WAVES 4
#endif
constexpr int kQuadBlockWaves = PCRIT_QUAD_BLOCK_WAVES;  // waves sharing one copy of the tables
struct QuadArgs {
  const float *f;        // full-resolution field
  int64_t fbytes;        // its size in bytes (loads past it read zeros)
  uint8_t *codes;        // full-resolution code bytes, or null
  const uint8_t *lut;    // quad table (device, kQuadTableSize bytes)
  LevelDesc lv;
  unsigned *nan_flag;
  unsigned gen;
  // Region timeline (null unless requested): the waves of XCD x take the
  // tiles of tile_list[xcd_off[x] ..] in order, one at a time, through the
  // counter queue[kCounterStride x] (zero at launch); a tile belongs to
  // region (rz, ry) of edge region_edge (full-resolution rows and planes);
  // the wave that finishes a region's last tile (region_left[kCounterStride
  // r] counts down) stores the GPU clock in region_stamp[r].
  const int *tile_list;
  const int *xcd_off;
  int *queue;
  unsigned *region_left;
  uint64_t *region_stamp;
  int region_edge, nry;
};
// Level geometry of a quad launch; whether a level can take one (stride 1
// or 2, 16-byte aligned rows).
// zmax > 0: the depth is also a power of two that is at most zmax.
void plan_level_quad(LevelDesc &l, int zmax = 0);
bool quad_eligible(const float *field, int64_t nx, int64_t s, int dim);
hipError_t launch_classify_quad(const QuadArgs &a, hipStream_t st);

// Fixed scratch of the allocation-free entry point (one copy per GPU):
// critical bitmask words, then per-chunk counts at a 256-byte boundary.
constexpr int64_t kNoAllocScratchBytes = int64_t(32) << 20;
hipError_t noalloc_scratch_init(int device);  // with `device` current
void *noalloc_scratch(int device);            // null before the init

// Learned refinement order (learned.hip).  MLP parameters, FP32, in this
// order: W1 [32 inputs][64], b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
constexpr int kMlpIn = 32, kMlpHidden = 64;
constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpIn * kMlpHidden;
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpHidden * kMlpHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpHidden;
constexpr int kMlpParams = kMlpOffB3 + 1;
constexpr int kMaxRegions = 1024;
hipError_t launch_mlp_forward(const float *params, const uint16_t *X, int64_t n, float *logits,
                              hipStream_t st);
hipError_t launch_mlp_backward(const float *params, const uint16_t *X, const uint8_t *y,
                               int64_t n, float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, float lr,
                           int t, hipStream_t st);
hipError_t launch_mlp_features(const float *f, int64_t nx, int64_t ny, int64_t nz, int s,
                               int mx, int my, int mz, float res, uint16_t *X, hipStream_t st);
hipError_t launch_mlp_labels(const uint8_t *codes, int64_t nx, int64_t ny, int64_t nz, int s,
                             int mx, int my, int mz, uint8_t *label, hipStream_t st);
// Region ranks from scores[stride r] (descending score, then ascending
// region id).
hipError_t launch_region_rank(const float *scores, int stride, int nregions, int *rank,
                              hipStream_t st);
// Region scores of the learned order straight from the field (inputs of
// level stride s, network, sigmoid, per-region sums): scores[kCounterStride
// r], kCounterStride * nregions floats, overwritten.
hipError_t launch_mlp_region_scores(const float *params, const float *f, int64_t nx, int64_t ny,
                                    int s, int mx, int my, int mz, float res, int E, int nry,
                                    int nregions, float *scores, hipStream_t st);
// Tile lists of a quad level for its region-ordered launch, and each
// region's tile count in region_left[kCounterStride r].  The tiles of every region are split
// into kXcds contiguous parts; list x (at xcd_off[x] .. xcd_off[x + 1] of
// tile_list) holds part x of every region, regions in rank order, and is
// drained in that order by the workgroups of XCD x (blockIdx.x % kXcds)
// through the counter queue[kCounterStride x].  scratch:
// kRegionScratchInts(nregions) ints; xcd_off and queue point into it
// (region_xcd_off, region_queue).  Counters that many waves update sit
// kCounterStride ints (256 bytes) apart: device-scope atomics on one line
// from every XCD serialise.
constexpr int kXcds = 8;
constexpr int kCounterStride = 64;
__host__ __device__ constexpr int64_t kRegionScratchInts(int nregions) {
  return 16 + kCounterStride * kXcds + (int64_t)kXcds * nregions;
}
__host__ __device__ inline int *region_xcd_off(int *scratch, int) { return scratch; }
__host__ __device__ inline int *region_queue(int *scratch, int) { return scratch + 16; }
// where part x of the region at rank k starts in list x: [kXcds k + x]
__host__ __device__ inline int *region_part_start(int *scratch, int) {
  return scratch + 16 + kCounterStride * kXcds;
}
hipError_t launch_region_tiles(const LevelDesc &l, int R, int s, int E, int nry, int nregions,
                               const int *rank, int *tile_list, unsigned *region_left,
                               int *scratch, hipStream_t st);
// Stores the GPU clock (100 MHz) in *out.
hipError_t launch_stamp(uint64_t *out, hipStream_t st);
// Zeroes n int64 values with a kernel (a memset node misbehaves in captured
// graphs).
hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t st);

// Order field (order.hip): rank[i] of every sample by (value, index) and the
// sample at each rank (sorted, also the sort's value buffer); scratch of
// order_scratch_bytes(n) bytes; a NaN sample sets *nan_flag = gen.
int64_t order_scratch_bytes(int64_t n);
hipError_t launch_order_field(const float *f, int64_t n, uint32_t *rank, uint32_t *sorted,
                              void *scratch, unsigned *nan_flag, unsigned gen, hipStream_t st);
// Minimum and maximum bits of full-resolution codes: rows * rowwords words
// of minima, then as many of maxima.
hipError_t launch_extrema_bits(const uint8_t *codes, int64_t nx, int64_t rows, int rowwords,
                               uint64_t *bits, hipStream_t st);
// Waits about `us` microseconds on the GPU, then stores the clock in *out.
hipError_t launch_wait_stamp(uint64_t *out, double us, hipStream_t st);

}  // namespace pcrit
