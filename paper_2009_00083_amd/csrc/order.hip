// Order field and extremum lists (gfx950).
//
// The order field (Section 4.1) ranks every vertex by (value, memory index):
// equal values are ordered by their index, so the ranks are a permutation.
// Here it is a least-significant-digit radix sort of 32-bit keys that order
// like the float values (sign-flipped bit patterns, -0 folded onto +0), with
// the vertex indices as values: a stable sort of keys that start in index
// order leaves equal keys in index order, which is exactly the tie-break.
// Four passes of 8 bits, each three kernels: per-tile digit histograms, one
// exclusive scan over (digit, tile), and a stable scatter that sorts each
// tile by digit in LDS (wave ballots on the digit's bits, per-wave digit
// counts) and writes its digit runs at their offsets.
// Finally rank[sorted[i]] = i.
//
// The extremum lists (the minima and maxima the paper's simplification
// starts from) are the vertices whose lower (upper) link is empty: bits
// from the level-0 codes, compacted by the library's list compaction.
#include <stdint.h>

#include <utility>

#include "device_util.h"
#include "pcrit_internal.h"

namespace pcrit {
namespace {

using namespace dev;

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 16;                       // keys per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys
constexpr int kRadix = 256;
static_assert(kSortThreads == kRadix, "one thread per digit in the tile kernels");

// Key whose unsigned order is the float order, -0 and +0 equal.
__device__ __forceinline__ uint32_t order_key(float v) {
  uint32_t b = __float_as_uint(v);
  if ((b & 0x7FFFFFFFu) == 0u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Keys of every sample and the identity permutation; NaN sets the flag.
__global__ void order_keys_kernel(const float *f, uint32_t n, uint32_t *keys, uint32_t *vals,
                                  unsigned *nan_flag, unsigned gen) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = f[i];
  if (v != v) *nan_flag = gen;
  keys[i] = order_key(v);
  vals[i] = i;
}

// hist[d * ntiles + t] = keys of tile t whose digit (bits shift .. shift+7)
// is d.
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t *keys, uint32_t n,
                                                                  int shift, uint32_t ntiles,
                                                                  uint32_t *hist) {
  __shared__ uint32_t s_h[kRadix];
  const int tid = threadIdx.x;
  s_h[tid] = 0u;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    const uint64_t i = base + (uint64_t)k * kSortThreads + tid;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(uint64_t)tid * ntiles + blockIdx.x] = s_h[tid];
}

// Exclusive scan of m values in place, three steps: sums of chunks of
// kSortTile values, a scan of the chunk sums (one block), and the chunks
// scanned from their offsets.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_w,
                                                         uint32_t *total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); i++) {
    before += i < w ? s_w[i] : 0u;
    all += s_w[i];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kSortThreads) void scan_chunk_sums_kernel(const uint32_t *a,
                                                                       uint64_t m,
                                                                       uint32_t *sums) {
  __shared__ uint32_t s_w[kSortWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)threadIdx.x * kSortItems;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kSortItems; k++) acc += base + k < m ? a[base + k] : 0u;
  uint32_t total;
  block_exclusive_scan(acc, s_w, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(uint32_t *sums, uint32_t nchunks) {
  __shared__ uint32_t s_w[16];
  // each thread scans a contiguous run of the chunk sums
  const uint32_t per = (nchunks + blockDim.x - 1) / blockDim.x;
  const uint32_t b = threadIdx.x * per, e = min(b + per, nchunks);
  uint32_t acc = 0;
  for (uint32_t i = b; i < e; i++) acc += sums[i];
  uint32_t total;
  uint32_t run = block_exclusive_scan(acc, s_w, &total);
  for (uint32_t i = b; i < e; i++) {
    const uint32_t v = sums[i];
    sums[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(kSortThreads) void scan_chunks_kernel(uint32_t *a, uint64_t m,
                                                                   const uint32_t *sums) {
  __shared__ uint32_t s_w[kSortWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)threadIdx.x * kSortItems;
  uint32_t v[kSortItems], acc = 0;
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    v[k] = base + k < m ? a[base + k] : 0u;
    acc += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(acc, s_w, &total) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    if (base + k < m) a[base + k] = run;
    run += v[k];
  }
}

// Stable scatter of tile t: key i of the tile goes to
// offset[d * ntiles + t] + (keys of digit d before it in the tile).  The
// tile's keys are first placed in LDS in digit order (a stable local sort:
// the tile is taken in rounds of kSortThreads keys, thread order = index
// order; within a wave the lanes with the same digit are found by ballots
// on its 8 bits, across waves and rounds by counts per digit in LDS), then
// written out in that order, so that consecutive threads write consecutive
// positions of a digit's run.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t *keys, const uint32_t *vals, uint32_t n, int shift, uint32_t ntiles,
    const uint32_t *offset, uint32_t *keys_out, uint32_t *vals_out) {
  __shared__ uint32_t s_key[kSortTile], s_val[kSortTile];
  __shared__ uint32_t s_lpre[kRadix];              // tile-local start of each digit
  __shared__ uint32_t s_run[kRadix];               // keys of each digit placed so far
  __shared__ uint32_t s_gbase[kRadix];             // global start of each digit
  __shared__ uint32_t s_wcnt[kSortWaves][kRadix];  // keys per wave and digit in a round
  __shared__ uint32_t s_w[kSortWaves];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const uint32_t cnt = (uint32_t)min((uint64_t)kSortTile, (uint64_t)n - base);
  uint32_t key[kSortItems], val[kSortItems];
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    const uint32_t j = (uint32_t)k * kSortThreads + tid;
    key[k] = j < cnt ? keys[base + j] : 0u;
    val[k] = j < cnt ? vals[base + j] : 0u;
  }
  s_run[tid] = 0u;
  s_gbase[tid] = offset[(uint64_t)tid * ntiles + blockIdx.x];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortItems; k++)
    if ((uint32_t)k * kSortThreads + tid < cnt) atomicAdd(&s_run[(key[k] >> shift) & 0xFFu], 1u);
  __syncthreads();
  uint32_t total;
  s_lpre[tid] = block_exclusive_scan(s_run[tid], s_w, &total);
  s_run[tid] = 0u;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes below this one
#pragma unroll
  for (int k = 0; k < kSortItems; k++) {
    for (int i = tid; i < kSortWaves * kRadix; i += kSortThreads) (&s_wcnt[0][0])[i] = 0u;
    __syncthreads();
    const bool ok = (uint32_t)k * kSortThreads + tid < cnt;
    const uint32_t d = (key[k] >> shift) & 0xFFu;
    uint64_t peers = wave_ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const uint64_t m = wave_ballot(((d >> b) & 1u) != 0u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t wrank = (uint32_t)__popcll(peers & lt);
    // the lowest lane of each digit group publishes the group's size
    if (ok && (peers & lt) == 0ull) s_wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (ok) {
      uint32_t pos = s_lpre[d] + s_run[d] + wrank;
      for (int v = 0; v < w; v++) pos += s_wcnt[v][d];
      s_key[pos] = key[k];
      s_val[pos] = val[k];
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int v = 0; v < kSortWaves; v++) sum += s_wcnt[v][tid];
    s_run[tid] += sum;
  }
  __syncthreads();
  for (uint32_t j = tid; j < cnt; j += kSortThreads) {
    const uint32_t kk = s_key[j], d = (kk >> shift) & 0xFFu;
    const uint32_t g = s_gbase[d] + (j - s_lpre[d]);
    keys_out[g] = kk;
    vals_out[g] = s_val[j];
  }
}

__global__ void rank_kernel(const uint32_t *sorted, uint32_t n, uint32_t *rank) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = sorted[i];
  if (v < n) rank[v] = i;  // a permutation of [0, n); the test keeps stray values out
}

// Minimum / maximum bits of level-0 codes, one 64-column word per thread:
// words [0, rows * rowwords) minima, then as many maxima.
__global__ void extrema_bits_kernel(const uint8_t *codes, int64_t nx, int64_t rows, int rowwords,
                                    uint64_t *bits) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * rowwords) return;
  const int64_t r = t / rowwords;
  const int xw = (int)(t - r * rowwords);
  const uint8_t *row = codes + r * nx;
  uint64_t mn = 0, mx = 0;
  const int x0 = 64 * xw, x1 = (int)min((int64_t)x0 + 64, nx);
  for (int x = x0; x < x1; x++) {
    const unsigned c = row[x];
    mn |= (uint64_t)((c & 7u) == 0u) << (x - x0);
    mx |= (uint64_t)((c & 0x38u) == 0u) << (x - x0);
  }
  bits[t] = mn;
  bits[rows * rowwords + t] = mx;
}

}  // namespace

int64_t order_scratch_bytes(int64_t n) {
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  const int64_t m = ntiles * kRadix;
  const int64_t nchunks = (m + kSortTile - 1) / kSortTile;
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  return 3 * up(4 * n) + up(4 * m) + up(4 * nchunks);
}

hipError_t launch_order_field(const float *f, int64_t n64, uint32_t *rank, uint32_t *sorted,
                              void *scratch, unsigned *nan_flag, unsigned gen, hipStream_t st) {
  const uint32_t n = (uint32_t)n64;
  const uint32_t ntiles = (uint32_t)((n64 + kSortTile - 1) / kSortTile);
  const uint64_t m = (uint64_t)ntiles * kRadix;
  const uint32_t nchunks = (uint32_t)((m + kSortTile - 1) / kSortTile);
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  char *p = static_cast<char *>(scratch);
  uint32_t *ka = reinterpret_cast<uint32_t *>(p);
  uint32_t *kb = reinterpret_cast<uint32_t *>(p + up(4 * n64));
  uint32_t *va = reinterpret_cast<uint32_t *>(p + 2 * up(4 * n64));
  uint32_t *hist = reinterpret_cast<uint32_t *>(p + 3 * up(4 * n64));
  uint32_t *sums = reinterpret_cast<uint32_t *>(p + 3 * up(4 * n64) + up(4 * (int64_t)m));
  // the values ping-pong between va and the caller's sorted array, which
  // holds them after the fourth pass
  uint32_t *vb = sorted;
  const unsigned g1 = (unsigned)((n64 + 255) / 256);
  hipLaunchKernelGGL(order_keys_kernel, dim3(g1), dim3(256), 0, st, f, n, ka, vb, nan_flag, gen);
  uint32_t *kin = ka, *kout = kb, *vin = vb, *vout = va;
  for (int pass = 0; pass < 4; pass++) {
    const int shift = 8 * pass;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(kSortThreads), 0, st, kin, n, shift,
                       ntiles, hist);
    hipLaunchKernelGGL(scan_chunk_sums_kernel, dim3(nchunks), dim3(kSortThreads), 0, st, hist, m,
                       sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, sums, nchunks);
    hipLaunchKernelGGL(scan_chunks_kernel, dim3(nchunks), dim3(kSortThreads), 0, st, hist, m,
                       sums);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(kSortThreads), 0, st, kin, vin, n,
                       shift, ntiles, hist, kout, vout);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  // four passes: the values are back in vb = sorted
  hipLaunchKernelGGL(rank_kernel, dim3(g1), dim3(256), 0, st, sorted, n, rank);
  return hipGetLastError();
}

hipError_t launch_extrema_bits(const uint8_t *codes, int64_t nx, int64_t rows, int rowwords,
                               uint64_t *bits, hipStream_t st) {
  const int64_t words = rows * rowwords;
  hipLaunchKernelGGL(extrema_bits_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                     codes, nx, rows, rowwords, bits);
  return hipGetLastError();
}

}  // namespace pcrit
