// C ABI of the classifier: argument checks, level geometry, scratch, the
// direct and the progressive drivers.  Every step of the classification runs
// in the kernels of classify.hip; this file only validates, sizes and
// enqueues.
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "../../include/pcrit.h"
#include "pcrit_internal.h"

using namespace pcrit;

namespace {

constexpr int kMaxLevels = 40;

struct Geom {
  int dim = 0;
  int64_t nx = 0, ny = 0, nz = 0;
  int level = 0;
  int64_t s = 1;
  int64_t mx = 0, my = 0, mz = 0;
  int64_t rowwords = 0, rows = 0, words = 0;
};

int check_dims(int64_t nx, int64_t ny, int64_t nz) {
  if (nx < 2 || ny < 2 || nz < 1) return PCRIT_E_DIMS;
  if (nx > 0xFFFFFFFFll || ny > 0xFFFFFFFFll || nz > 0xFFFFFFFFll)
    return PCRIT_E_DIMS;
  const double n = (double)nx * (double)ny * (double)nz;
  if (n > 4294967295.0) return PCRIT_E_DIMS;
  return PCRIT_OK;
}

int max_level_of(int64_t nx, int64_t ny, int64_t nz) {
  int64_t lim = std::min(nx, ny) - 1;
  if (nz > 1) lim = std::min(lim, nz - 1);
  int k = 0;
  while (k + 1 < kMaxLevels && ((int64_t)1 << (k + 1)) <= lim) k++;
  return k;
}

int make_geom(int64_t nx, int64_t ny, int64_t nz, int level, Geom *g) {
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  if (level < 0 || level > max_level_of(nx, ny, nz)) return PCRIT_E_LEVEL;
  g->dim = nz == 1 ? 2 : 3;
  g->nx = nx;
  g->ny = ny;
  g->nz = nz;
  g->level = level;
  g->s = (int64_t)1 << level;
  g->mx = (nx - 1) / g->s + 1;
  g->my = (ny - 1) / g->s + 1;
  g->mz = g->dim == 3 ? (nz - 1) / g->s + 1 : 1;
  g->rowwords = (g->mx + 63) / 64;
  g->rows = g->my * g->mz;
  g->words = g->rows * g->rowwords;
  return PCRIT_OK;
}

bool misaligned(const void *p, size_t a) {
  return ((uintptr_t)p & (a - 1)) != 0;
}

}  // namespace

struct pcrit_ctx {
  int device = 0;
  uint8_t *lut3 = nullptr, *lut2 = nullptr;
  uint64_t *bits[2] = {nullptr, nullptr};
  int64_t bits_words = 0;
  int *counts = nullptr;  // per-chunk critical counts of the compaction
  int64_t counts_n = 0;
  void *masks[2] = {nullptr, nullptr};  // polarity masks, level ping-pong
  int64_t masks_bytes = 0;
  unsigned *reclass_part = nullptr;  // per-block counts of a progressive level
  int reclass_n = 0;
  // One device status block read back with a single copy: level_base
  // (kMaxLevels + 2 list offsets, [0] stays 0) followed by flags ([0] nan,
  // [3 + i] re-classified old vertices of progressive step i).
  void *status = nullptr;
  int64_t *level_base = nullptr;
  unsigned *flags = nullptr;
  void *h_status = nullptr;  // pinned host mirror
  int64_t *h_base = nullptr;
  unsigned *h_flags = nullptr;
  unsigned gen = 0;
  uint64_t timing = 0;  // bit k: time the kernels of level k
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_level[kMaxLevels + 1] = {};
  hipEvent_t kev[2][kMaxLevels][2] = {};
  bool kused[2][kMaxLevels] = {};
  hipEvent_t last_kev = nullptr;
};

namespace {

constexpr int kFlagWords = 3 + kMaxLevels + 2;
constexpr size_t kStatusBytes =
    (kMaxLevels + 2) * sizeof(int64_t) + kFlagWords * sizeof(unsigned);

// Copy the status block to the host and wait for the stream.
int read_status(pcrit_ctx *c, hipStream_t s) {
  if (hipMemcpyAsync(c->h_status, c->status, kStatusBytes,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PCRIT_E_HIP;
  return PCRIT_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? PCRIT_OK : PCRIT_E_HIP; }

int ensure_masks(pcrit_ctx *c, int64_t bytes) {
  if (bytes <= c->masks_bytes) return PCRIT_OK;
  hipDeviceSynchronize();
  for (int i = 0; i < 2; i++) {
    if (c->masks[i]) hipFree(c->masks[i]);
    c->masks[i] = nullptr;
  }
  c->masks_bytes = 0;
  for (int i = 0; i < 2; i++)
    if (hipMalloc(&c->masks[i], (size_t)bytes) != hipSuccess) return PCRIT_E_OOM;
  c->masks_bytes = bytes;
  return PCRIT_OK;
}

int ensure_scratch(pcrit_ctx *c, int64_t words, int64_t chunks) {
  if (words > c->bits_words) {
    hipDeviceSynchronize();
    for (int i = 0; i < 2; i++) {
      if (c->bits[i]) hipFree(c->bits[i]);
      c->bits[i] = nullptr;
    }
    c->bits_words = 0;
    for (int i = 0; i < 2; i++)
      if (hipMalloc(&c->bits[i], (size_t)words * 8) != hipSuccess)
        return PCRIT_E_OOM;
    c->bits_words = words;
  }
  if (chunks > c->counts_n) {
    hipDeviceSynchronize();
    if (c->counts) hipFree(c->counts);
    c->counts = nullptr;
    c->counts_n = 0;
    if (hipMalloc(&c->counts, (size_t)chunks * sizeof(int)) != hipSuccess)
      return PCRIT_E_OOM;
    c->counts_n = chunks;
  }
  return PCRIT_OK;
}

unsigned next_gen(pcrit_ctx *c) {
  if (++c->gen == 0) c->gen = 1;
  return c->gen;
}

void record_kernel(pcrit_ctx *c, int which, int level, int end, hipStream_t st) {
  if (level < 0 || level >= kMaxLevels || !((c->timing >> level) & 1)) return;
  hipEvent_t &e = c->kev[which][level][end];
  if (!e) hipEventCreate(&e);
  hipEventRecord(e, st);
  c->kused[which][level] = true;
  if (end) c->last_kev = e;
}

// Enqueue classification (+ compaction) of one level.
// Progressive steps: prev != null reads the polarity masks of the previous
// (coarser) level from masks[mask_slot ^ 1]; write_masks stores this level's
// masks into masks[mask_slot] for the next level.
int enqueue_level(pcrit_ctx *c, hipStream_t st, const float *field,
                  const Geom &g, const Geom *prev, bool write_masks,
                  int bits_out, int mask_slot, uint8_t *codes, uint32_t *crit,
                  uint8_t *crit_codes, int64_t cap, int slot,
                  int64_t *count_dev, unsigned gen, unsigned *reclass) {
  const bool progressive = prev != nullptr;
  const int64_t chunks = (g.words + kChunkWords - 1) / kChunkWords;
  ClassifyArgs a{};
  a.f = field;
  a.codes = codes;
  a.bits = c->bits[bits_out];
  a.lut = g.dim == 3 ? c->lut3 : c->lut2;
  a.sx = g.s;
  a.sy = g.s * g.nx;
  a.sz = g.s * g.nx * g.ny;
  a.mx = (int)g.mx;
  a.my = (int)g.my;
  a.mz = (int)g.mz;
  a.rowwords = (int)g.rowwords;
  if (progressive) {
    a.prev_masks = c->masks[mask_slot ^ 1];
    a.pmx = (int)prev->mx;
    a.pmy = (int)prev->my;
  }
  if (write_masks) a.masks = c->masks[mask_slot];
  a.reclass_part = c->reclass_part;
  a.nan_flag = &c->flags[0];
  a.gen = gen;
  hipError_t e;
  int grid = 0;
  record_kernel(c, 0, g.level, 0, st);
  if (g.dim == 3)
    e = launch_classify3d(a, progressive, write_masks, st, &grid);
  else
    e = launch_classify2d(a, progressive, write_masks, st, &grid);
  if (e != hipSuccess) return PCRIT_E_HIP;
  record_kernel(c, 0, g.level, 1, st);

  CompactArgs b{};
  b.bits = c->bits[bits_out];
  b.words = g.words;
  b.rowwords = (int)g.rowwords;
  b.my = (int)g.my;
  b.s = g.s;
  b.nx = g.nx;
  b.ny = g.ny;
  b.crit = crit;
  b.crit_codes = crit_codes;
  b.codes = codes;
  b.cap = cap;
  b.level_base = c->level_base;
  b.slot = slot;
  b.count_dev = count_dev;
  b.nan_flag = &c->flags[0];
  b.gen = gen;
  b.counts = c->counts;
  b.nchunks = (int)chunks;
  if (progressive) {
    b.reclass_part = c->reclass_part;
    b.reclass_n = std::min(grid, c->reclass_n);
    b.reclass_out = reclass;
  }
  record_kernel(c, 1, g.level, 0, st);
  e = launch_compact(b, st);
  if (e != hipSuccess) return PCRIT_E_HIP;
  record_kernel(c, 1, g.level, 1, st);
  return PCRIT_OK;
}

void reset_kernel_marks(pcrit_ctx *c) {
  memset(c->kused, 0, sizeof(c->kused));
  c->last_kev = nullptr;
}

}  // namespace

extern "C" {

const char *pcrit_strerror(int status) {
  switch (status) {
    case PCRIT_OK: return "ok";
    case PCRIT_E_ARG: return "invalid argument (null or misaligned pointer, bad value)";
    case PCRIT_E_DIMS: return "invalid grid dimensions";
    case PCRIT_E_LEVEL: return "level outside the hierarchy of this grid";
    case PCRIT_E_CAPACITY: return "critical list capacity too small";
    case PCRIT_E_NAN: return "NaN sample in the field";
    case PCRIT_E_HIP: return "HIP runtime error";
    case PCRIT_E_OOM: return "device allocation failed";
    default: return "unknown status";
  }
}

int pcrit_max_level(int64_t nx, int64_t ny, int64_t nz, int *k_max_host) {
  if (!k_max_host) return PCRIT_E_ARG;
  const int st = check_dims(nx, ny, nz);
  if (st) return st;
  *k_max_host = max_level_of(nx, ny, nz);
  return PCRIT_OK;
}

int pcrit_level_dims(int64_t nx, int64_t ny, int64_t nz, int level,
                     int64_t *m3_host) {
  if (!m3_host) return PCRIT_E_ARG;
  Geom g;
  const int st = make_geom(nx, ny, nz, level, &g);
  if (st) return st;
  m3_host[0] = g.mx;
  m3_host[1] = g.my;
  m3_host[2] = g.mz;
  return PCRIT_OK;
}

int pcrit_link_table(int dim, uint8_t *table_host, int64_t size) {
  if (!table_host) return PCRIT_E_ARG;
  if (dim == 3 && size >= kLut3Size) {
    build_link_table3(table_host);
    return PCRIT_OK;
  }
  if (dim == 2 && size >= kLut2Size) {
    build_link_table2(table_host);
    return PCRIT_OK;
  }
  return PCRIT_E_ARG;
}

int pcrit_create(pcrit_ctx **out, int hip_device) {
  if (!out) return PCRIT_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 ||
      hip_device >= ndev)
    return PCRIT_E_HIP;
  if (hipSetDevice(hip_device) != hipSuccess) return PCRIT_E_HIP;
  pcrit_ctx *c = new pcrit_ctx();
  c->device = hip_device;
  c->reclass_n = classify_max_blocks();
  uint8_t h3[kLut3Size], h2[kLut2Size];
  build_link_table3(h3);
  build_link_table2(h2);
  bool ok = hipMalloc(&c->lut3, kLut3Size) == hipSuccess &&
            hipMalloc(&c->lut2, kLut2Size) == hipSuccess &&
            hipMalloc(&c->status, kStatusBytes) == hipSuccess &&
            hipMalloc(&c->reclass_part, classify_max_blocks() * sizeof(unsigned)) ==
                hipSuccess &&
            hipHostMalloc(&c->h_status, kStatusBytes) == hipSuccess;
  if (ok) {
    c->level_base = (int64_t *)c->status;
    c->flags = (unsigned *)((char *)c->status + (kMaxLevels + 2) * sizeof(int64_t));
    c->h_base = (int64_t *)c->h_status;
    c->h_flags = (unsigned *)((char *)c->h_status + (kMaxLevels + 2) * sizeof(int64_t));
  }
  ok = ok && hipMemcpy(c->lut3, h3, kLut3Size, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(c->lut2, h2, kLut2Size, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(c->status, 0, kStatusBytes) == hipSuccess;
  ok = ok && hipEventCreate(&c->ev_start) == hipSuccess;
  for (int i = 0; ok && i <= kMaxLevels; i++)
    ok = hipEventCreate(&c->ev_level[i]) == hipSuccess;
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    pcrit_destroy(c);
    return PCRIT_E_OOM;
  }
  *out = c;
  return PCRIT_OK;
}

void pcrit_destroy(pcrit_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  hipFree(c->lut3);
  hipFree(c->lut2);
  hipFree(c->bits[0]);
  hipFree(c->bits[1]);
  hipFree(c->counts);
  hipFree(c->masks[0]);
  hipFree(c->masks[1]);
  hipFree(c->reclass_part);
  hipFree(c->status);
  if (c->h_status) hipHostFree(c->h_status);
  if (c->ev_start) hipEventDestroy(c->ev_start);
  for (int i = 0; i <= kMaxLevels; i++)
    if (c->ev_level[i]) hipEventDestroy(c->ev_level[i]);
  for (int w = 0; w < 2; w++)
    for (int l = 0; l < kMaxLevels; l++)
      for (int e = 0; e < 2; e++)
        if (c->kev[w][l][e]) hipEventDestroy(c->kev[w][l][e]);
  delete c;
}

int pcrit_classify(pcrit_ctx *c, void *hip_stream, const float *field,
                   int64_t nx, int64_t ny, int64_t nz, int level,
                   uint8_t *codes, uint32_t *crit, uint8_t *crit_codes,
                   int64_t crit_capacity, int64_t *crit_count_host,
                   int64_t *crit_count_dev) {
  if (!c || !field || !codes || crit_capacity < 0 ||
      (crit_capacity > 0 && !crit))
    return PCRIT_E_ARG;
  if (misaligned(field, 4) || (crit && misaligned(crit, 4)) ||
      (crit_count_dev && misaligned(crit_count_dev, 8)))
    return PCRIT_E_ARG;
  Geom g;
  int st = make_geom(nx, ny, nz, level, &g);
  if (st) return st;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  st = ensure_scratch(c, g.words, (g.words + kChunkWords - 1) / kChunkWords);
  if (st) return st;
  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  st = enqueue_level(c, s, field, g, nullptr, false, 0, 0, codes, crit,
                     crit_codes, crit_capacity, 0, crit_count_dev, gen,
                     nullptr);
  if (st) return st;
  if (!crit_count_host) return PCRIT_OK;
  if (read_status(c, s)) return PCRIT_E_HIP;
  const int64_t count = c->h_base[1] - c->h_base[0];
  *crit_count_host = count;
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return count > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

int pcrit_progressive(pcrit_ctx *c, void *hip_stream, const float *field,
                      int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                      uint32_t *crit, uint8_t *crit_codes,
                      int64_t crit_capacity, int64_t *level_offsets_host,
                      float *level_ms_host, int64_t *reclassified_host,
                      pcrit_level_cb cb, void *user) {
  if (!c || !field || !codes || crit_capacity < 0 ||
      (crit_capacity > 0 && !crit))
    return PCRIT_E_ARG;
  if (misaligned(field, 4) || (crit && misaligned(crit, 4)))
    return PCRIT_E_ARG;
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int kmax = max_level_of(nx, ny, nz);
  Geom geo[kMaxLevels];
  for (int k = 0; k <= kmax; k++) {
    st = make_geom(nx, ny, nz, k, &geo[k]);
    if (st) return st;
  }
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  int64_t max_words = 0;
  for (int k = 0; k <= kmax; k++) max_words = std::max(max_words, geo[k].words);
  st = ensure_scratch(c, max_words, (max_words + kChunkWords - 1) / kChunkWords);
  if (st) return st;
  if (kmax > 0) {
    // masks of levels kmax .. 1 (the finest of them is the largest)
    const Geom &g1 = geo[1];
    st = ensure_masks(c, g1.mx * g1.my * g1.mz * (g1.dim == 3 ? 2 : 1));
    if (st) return st;
  }
  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  if (hipEventRecord(c->ev_start, s) != hipSuccess) return PCRIT_E_HIP;
  for (int i = 0; i <= kmax; i++) {
    const int k = kmax - i;
    st = enqueue_level(c, s, field, geo[k], i > 0 ? &geo[k + 1] : nullptr,
                       k > 0, i & 1, i & 1, codes, crit, crit_codes,
                       crit_capacity, i, nullptr, gen, &c->flags[3 + i]);
    if (st) return st;
    if (hipEventRecord(c->ev_level[i], s) != hipSuccess) return PCRIT_E_HIP;
    if (cb) {
      if (read_status(c, s)) return PCRIT_E_HIP;
      cb(k, c->h_base[i + 1] - c->h_base[i], user);
    }
  }
  if (read_status(c, s)) return PCRIT_E_HIP;
  if (level_offsets_host)
    for (int i = 0; i <= kmax + 1; i++) level_offsets_host[i] = c->h_base[i];
  if (reclassified_host)
    for (int i = 0; i <= kmax; i++)
      reclassified_host[i] = i == 0 ? 0 : (int64_t)c->h_flags[3 + i];
  if (level_ms_host)
    for (int i = 0; i <= kmax; i++) {
      float ms = -1.f;
      if (hipEventElapsedTime(&ms, c->ev_start, c->ev_level[i]) != hipSuccess)
        ms = -1.f;
      level_ms_host[i] = ms;
    }
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return c->h_base[kmax + 1] > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

int pcrit_set_kernel_timing(pcrit_ctx *c, uint64_t level_mask) {
  if (!c) return PCRIT_E_ARG;
  c->timing = level_mask;
  return PCRIT_OK;
}

int pcrit_kernel_ms(pcrit_ctx *c, float *classify_ms_host,
                    float *compact_ms_host, int max_levels) {
  if (!c || max_levels < 0) return PCRIT_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  if (c->last_kev && hipEventSynchronize(c->last_kev) != hipSuccess)
    return PCRIT_E_HIP;
  float *outs[2] = {classify_ms_host, compact_ms_host};
  for (int w = 0; w < 2; w++) {
    if (!outs[w]) continue;
    for (int l = 0; l < max_levels; l++) {
      float ms = -1.f;
      if (l < kMaxLevels && c->kused[w][l] &&
          hipEventElapsedTime(&ms, c->kev[w][l][0], c->kev[w][l][1]) != hipSuccess)
        ms = -1.f;
      outs[w][l] = ms;
    }
  }
  return PCRIT_OK;
}

}  // extern "C"
