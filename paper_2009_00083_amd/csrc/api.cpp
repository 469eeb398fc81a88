// C ABI of the classifier: argument checks, level geometry, scratch, the
// direct and the progressive drivers.  Every step of the classification runs
// in the kernels of classify.hip; this file only validates, sizes and
// enqueues.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pcrit.h"
#include "batch_tune.h"
#include "pcrit_internal.h"
#include "lts.h"

using namespace pcrit;

static_assert(kNoAllocScratchBytes == PCRIT_NOALLOC_SCRATCH_BYTES,
              "scratch size of the header and of the library");
static_assert(kMlpParams == PCRIT_MLP_PARAMS && kMlpIn == PCRIT_MLP_INPUTS,
              "network size of the header and of the library");

namespace {

constexpr int kMaxLevels = 40;

struct Geom {
  int dim = 0;
  int64_t nx = 0, ny = 0, nz = 0;
  int level = 0;
  int64_t s = 1;
  int64_t mx = 0, my = 0, mz = 0;
  int64_t rowwords = 0, rows = 0, words = 0;
  bool quad = false;  // classified on quad tiles
};

void set_quad(Geom *g, bool quad) { g->quad = quad; }

int check_dims(int64_t nx, int64_t ny, int64_t nz) {
  if (nx < 2 || ny < 2 || nz < 1) return PCRIT_E_DIMS;
  if (nx > 0xFFFFFFFFll || ny > 0xFFFFFFFFll || nz > 0xFFFFFFFFll)
    return PCRIT_E_DIMS;
  const double n = (double)nx * (double)ny * (double)nz;
  if (n > 4294967295.0) return PCRIT_E_DIMS;
  // the kernels address a plane (3D) or a row (2D) through buffer
  // descriptors whose byte range ends at 2^32 - 1: at most 2^30 - 1 samples
  if ((nz > 1 ? (double)nx * (double)ny : (double)nx) > 1073741823.0)
    return PCRIT_E_DIMS;
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
  g->rowwords = (g->mx + kTileCols - 1) / kTileCols;
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
  uint8_t *lutq = nullptr;  // quad-tile tables (kQuadTableBytes bytes)
  uint64_t *bits = nullptr;  // critical bitmasks of the levels of one launch
  int64_t bits_words = 0;
  // the finest level's bitmask and chunk counts when it runs beside the
  // coarser levels (progressive calls, see enqueue_progressive)
  uint64_t *bits2 = nullptr;
  int64_t bits2_words = 0;
  int *counts2 = nullptr;
  int64_t counts2_n = 0;
  int *counts = nullptr;  // per-chunk critical counts of the compaction
  int64_t counts_n = 0;
  uint8_t *lcodes = nullptr;  // dense codes of fused levels (for crit_codes)
  int64_t lcodes_bytes = 0;
  void *masks[2] = {nullptr, nullptr};  // polarity masks, level ping-pong
  int64_t masks_bytes = 0;
  // Re-classified old vertices per level of a launch: the classification
  // adds to them, the compaction reads them and sets them back to zero.
  unsigned *reclass_acc = nullptr;
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
  void *tl = nullptr;  // region timeline and learned-order scratch
  int64_t tl_bytes = 0;
  int64_t *boff = nullptr;  // list offsets of a batch (when the caller gives none)
  int64_t boff_bytes = 0;
  void *ord = nullptr;  // order-field sort scratch
  int64_t ord_bytes = 0;
  void *lts = nullptr;  // merged-propagation records and saddle table
  int64_t lts_bytes = 0;
  // batch launches: fields per shared launch, wave tiles per field
  int batch_group = kBatchGroupDefault;
  int64_t batch_want = kBatchWantDefault;
  // second stream (default priority) on which the learned order is scored
  // while the leading levels run, and the events that fork and join it
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // batch pipeline: group g's classification done (ev_cls), its compaction
  // done (ev_cmp), per scratch set g % 2
  hipEvent_t ev_cls[2] = {}, ev_cmp[2] = {};
};

// GPU wait ahead of the first stamp or start event of a timed call
// (microseconds)
constexpr double kTimelineLeadUs = 300.0;

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

// Grow a scratch allocation (contents are not kept).
int ensure(void **p, int64_t *have, int64_t bytes) {
  if (bytes <= *have) return PCRIT_OK;
  hipDeviceSynchronize();
  if (*p) hipFree(*p);
  *p = nullptr;
  *have = 0;
  if (hipMalloc(p, (size_t)bytes) != hipSuccess) return PCRIT_E_OOM;
  *have = bytes;
  return PCRIT_OK;
}

// The context's second stream (default priority) and the events that fork
// work onto it and join it back.
int ensure_side(pcrit_ctx *c) {
  if (!c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
    c->side = nullptr;
    return PCRIT_E_HIP;
  }
  hipEvent_t *evs[6] = {&c->ev_fork, &c->ev_join, &c->ev_cls[0], &c->ev_cls[1],
                        &c->ev_cmp[0], &c->ev_cmp[1]};
  for (hipEvent_t *e : evs)
    if (!*e && hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
      *e = nullptr;
      return PCRIT_E_HIP;
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

// One level of a launch.
struct Step {
  Geom g;
  // batches: this step's own field and codes (else the call's), and every
  // step writes its codes
  const float *f = nullptr;
  uint8_t *codes = nullptr;
  bool batch = false;
  int64_t want = 0;  // batches: wave tiles per field (0: the launch's default)
  const Geom *prev = nullptr;  // previous (coarser) level, progressive only
  bool dirty = false;          // test old vertices against `prev`
  int mask_read = -1;          // masks slot holding prev's masks, or -1
  int mask_write = -1;         // masks slot for this level's masks, or -1
  int slot = 0;                // list slot (level_base index)
  unsigned *reclass_out = nullptr;
};

int64_t level_vertices(const Geom &g) { return g.mx * g.my * g.mz; }

// Scratch one launch of steps[0..n) needs.
void launch_needs(const Step *steps, int n, bool with_codes, int64_t *words,
                  int64_t *chunks, int64_t *lbytes) {
  const bool fused = n > 1;
  int64_t total = 0;
  for (int l = 0; l < n; l++) total += steps[l].g.words;
  const int64_t cw = small_chunks(total) ? kSmallChunkWords : kChunkWords;
  *words = *chunks = *lbytes = 0;
  for (int l = 0; l < n; l++) {
    *words += steps[l].g.words;
    *chunks += (steps[l].g.words + cw - 1) / cw;
    if (fused && l + 1 < n && with_codes) *lbytes += level_vertices(steps[l].g);
  }
}

// Enqueue classification + compaction of steps[0..n): one level, or several
// small levels fused into one launch of each kernel.  In a fused launch the
// levels run concurrently: old vertices are tested against the previous
// level's masks computed from the field, only the finest level stores its
// codes at full resolution (its vertices include those of the others), and
// the others keep dense level codes for crit_codes.
// `bits` and `counts` are the launch's scratch (the context's, or the fixed
// array of the allocation-free entry point).
// Region timeline of a quad level: tiles taken region by region in rank
// order, each region's completion stamped (see QuadArgs).
struct RegionHooks {
  int E = 0, nry = 0, nregions = 0;
  const int *rank = nullptr;  // device, per region
  int *tile_list = nullptr, *scratch = nullptr;
  unsigned *left = nullptr;
  uint64_t *stamp = nullptr;  // this level's row of region stamps
  bool prebuilt = false;      // tile lists already built (else built here)
};

int enqueue_group(pcrit_ctx *c, hipStream_t st, const float *field,
                  const Step *steps, int n, uint8_t *codes, uint32_t *crit,
                  uint8_t *crit_codes, int64_t cap, int64_t *count_dev,
                  unsigned gen, bool final_group, uint64_t *bits, int *counts,
                  int64_t *publish = nullptr, int publish_n = 0,
                  const RegionHooks *rh = nullptr, int64_t *lbase = nullptr,
                  hipEvent_t compact_after = nullptr, hipStream_t compact_st = nullptr,
                  hipEvent_t classified = nullptr) {
  const bool fused = n > 1;
  const int dim = steps[0].g.dim;
  int64_t total_words = 0;
  for (int l = 0; l < n; l++) total_words += steps[l].g.words;
  const bool small = small_chunks(total_words);
  const int64_t cw = small ? kSmallChunkWords : kChunkWords;
  ClassifyArgs a{};
  a.lut = dim == 3 ? c->lut3 : c->lut2;
  a.nl = n;
  a.reclass_acc = c->reclass_acc;
  a.nan_flag = &c->flags[0];
  a.gen = gen;
  CompactArgs b{};
  b.nl = n;
  int64_t woff = 0, loff = 0, chunks = 0;
  int tiles = 0;
  for (int l = 0; l < n; l++) {
    const Step &sp = steps[l];
    const Geom &g = sp.g;
    const bool last = l == n - 1;
    LevelDesc &d = a.lv[l];
    d.f = sp.f ? sp.f : field;
    d.codes = sp.codes ? sp.codes : codes;
    d.sx = g.s;
    d.sy = g.s * g.nx;
    d.sz = g.s * g.nx * g.ny;
    d.mx = (int)g.mx;
    d.my = (int)g.my;
    d.mz = (int)g.mz;
    d.rowwords = (int)g.rowwords;
    // batches run as fused launches too (their steps test no old vertices):
    // measured on 200 fields of 33..257 samples per axis, the fused
    // kernel's 8-plane tiles take 2.15 ms, the plain kernel's 24-plane tiles
    // 2.31 ms
    if (sp.want > 0 && dim == 3)
      plan_level3_want(d, fused || steps[0].mask_write >= 0, sp.want);
    else if (sp.want > 0)
      plan_level2_want(d, sp.want);
    else if (dim == 3)
      plan_level3(d, fused || steps[0].mask_write >= 0, fused);
    else
      plan_level2(d, fused);
    d.tile_begin = tiles;
    tiles += d.ntiles;
    d.bits = bits + woff;
    d.lcodes = fused && !last && crit_codes && !sp.batch ? c->lcodes + loff : nullptr;
    if (!fused && sp.mask_read >= 0) d.prev_masks = c->masks[sp.mask_read];
    if (sp.prev) {
      d.pmx = (int)sp.prev->mx;
      d.pmy = (int)sp.prev->my;
    }
    if (sp.mask_write >= 0) d.masks = c->masks[sp.mask_write];
    // full-resolution codes: the last level of the call writes every code
    // (a vertex's code at its finest level); earlier levels only when their
    // lists carry codes
    d.write_codes = sp.batch || ((!fused || last) && (final_group || crit_codes != nullptr));
    d.dirty = sp.dirty;

    CompactLevel &q = b.lv[l];
    q.codes = d.codes;
    q.nx = g.nx;
    q.ny = g.ny;
    q.bits = d.bits;
    q.words = g.words;
    q.rowwords = (int)g.rowwords;
    q.mx = (int)g.mx;
    q.my = (int)g.my;
    q.s = g.s;
    q.slot = sp.slot;
    q.chunk_begin = (int)chunks;
    q.lcodes = d.lcodes;
    q.reclass_out = sp.reclass_out;
    q.linear = g.s == 1 && g.mx == g.rowwords * 64;
    woff += g.words;
    if (d.lcodes) loff += level_vertices(g);
    chunks += (g.words + cw - 1) / cw;
  }
  a.ntiles = tiles;
  const int tlevel = steps[n - 1].g.level;  // a launch is timed as its finest level
  const Step &s0 = steps[0];
  // Full-resolution and stride-2 levels of 3D grids with 16-byte aligned
  // rows take the quad tiles, unless the launch stores or reads masks for
  // the re-classification count.
  const bool quad = !fused && s0.g.quad;
  record_kernel(c, 0, tlevel, 0, st);
  if (quad) {
    QuadArgs q{};
    q.f = field;
    q.fbytes = s0.g.nx * s0.g.ny * s0.g.nz * (int64_t)sizeof(float);
    q.codes = a.lv[0].write_codes ? codes : nullptr;
    q.lut = c->lutq;
    q.lv = a.lv[0];
    q.nan_flag = a.nan_flag;
    q.gen = gen;
    if (rh) {
      const int s = (int)s0.g.s;
      plan_level_quad(q.lv, std::min(kQuadZChunk, rh->E / s));
      if (!rh->prebuilt &&
          launch_region_tiles(q.lv, kQuadRows, s, rh->E, rh->nry, rh->nregions, rh->rank,
                              rh->tile_list, rh->left, rh->scratch, st) != hipSuccess)
        return PCRIT_E_HIP;
      q.tile_list = rh->tile_list;
      q.xcd_off = region_xcd_off(rh->scratch, rh->nregions);
      q.queue = region_queue(rh->scratch, rh->nregions);
      q.region_left = rh->left;
      q.region_stamp = rh->stamp;
      q.region_edge = rh->E;
      q.nry = rh->nry;
    } else {
      plan_level_quad(q.lv);
    }
    if (launch_classify_quad(q, st) != hipSuccess) return PCRIT_E_HIP;
  } else if (launch_classify(a, dim, !fused && s0.mask_read >= 0,
                             !fused && s0.mask_write >= 0, fused, st) != hipSuccess) {
    return PCRIT_E_HIP;
  }
  record_kernel(c, 0, tlevel, 1, st);

  b.nchunks = (int)chunks;
  b.crit = crit;
  b.crit_codes = crit_codes;
  b.cap = cap;
  b.level_base = lbase ? lbase : c->level_base;
  b.count_dev = count_dev;
  b.publish = publish;
  b.publish_n = publish_n;
  b.nan_flag = &c->flags[0];
  b.gen = gen;
  b.counts = counts;
  b.reclass_acc = c->reclass_acc;
  // the lists of earlier launches that ran on another stream come first
  if (compact_after && hipStreamWaitEvent(st, compact_after, 0) != hipSuccess)
    return PCRIT_E_HIP;
  // or the compaction runs on another stream once the classification is
  // done (`classified` recorded here)
  if (compact_st) {
    if (hipEventRecord(classified, st) != hipSuccess ||
        hipStreamWaitEvent(compact_st, classified, 0) != hipSuccess)
      return PCRIT_E_HIP;
    st = compact_st;
  }
  record_kernel(c, 1, tlevel, 0, st);
  if (launch_compact(b, small, st) != hipSuccess) return PCRIT_E_HIP;
  record_kernel(c, 1, tlevel, 1, st);
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
    case PCRIT_E_SCRATCH:
      return "level too large for the fixed scratch of the allocation-free entry point";
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
  // device address of this GPU's fixed scratch (pcrit_classify_noalloc)
  if (noalloc_scratch_init(hip_device) != hipSuccess) return PCRIT_E_HIP;
  pcrit_ctx *c = new pcrit_ctx();
  c->device = hip_device;
  // device tables are indexed by raw masks (true mask ^ kPos)
  uint8_t t3[kLut3Size], t2[kLut2Size], h3[kLut3Size], h2[kLut2Size];
  std::vector<uint8_t> hq(kQuadTableBytes);
  build_link_table3(t3);
  build_link_table2(t2);
  for (int i = 0; i < kLut3Size; i++) h3[i] = t3[i ^ kPos3];
  for (int i = 0; i < kLut2Size; i++) h2[i] = t2[i ^ kPos2];
  build_quad_table3(t3, hq.data());
  bool ok = hipMalloc(&c->lut3, kLut3Size) == hipSuccess &&
            hipMalloc(&c->lut2, kLut2Size) == hipSuccess &&
            hipMalloc(&c->lutq, kQuadTableBytes) == hipSuccess &&
            hipMalloc(&c->status, kStatusBytes) == hipSuccess &&
            hipMalloc(&c->reclass_acc, kMaxFused * sizeof(unsigned)) == hipSuccess &&
            hipHostMalloc(&c->h_status, kStatusBytes) == hipSuccess;
  if (ok) {
    c->level_base = (int64_t *)c->status;
    c->flags = (unsigned *)((char *)c->status + (kMaxLevels + 2) * sizeof(int64_t));
    c->h_base = (int64_t *)c->h_status;
    c->h_flags = (unsigned *)((char *)c->h_status + (kMaxLevels + 2) * sizeof(int64_t));
  }
  ok = ok && hipMemcpy(c->lut3, h3, kLut3Size, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(c->lut2, h2, kLut2Size, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(c->lutq, hq.data(), kQuadTableBytes, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemset(c->status, 0, kStatusBytes) == hipSuccess &&
       hipMemset(c->reclass_acc, 0, kMaxFused * sizeof(unsigned)) == hipSuccess;
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
  hipFree(c->lutq);
  hipFree(c->bits);
  hipFree(c->counts);
  hipFree(c->bits2);
  hipFree(c->counts2);
  hipFree(c->lcodes);
  hipFree(c->masks[0]);
  hipFree(c->masks[1]);
  hipFree(c->reclass_acc);
  hipFree(c->tl);
  hipFree(c->boff);
  hipFree(c->ord);
  hipFree(c->lts);
  hipFree(c->status);
  if (c->side) hipStreamDestroy(c->side);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  for (int k = 0; k < 2; k++) {
    if (c->ev_cls[k]) hipEventDestroy(c->ev_cls[k]);
    if (c->ev_cmp[k]) hipEventDestroy(c->ev_cmp[k]);
  }
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
  set_quad(&g, quad_eligible(field, nx, g.s, g.dim));
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  Step step;
  step.g = g;
  int64_t words, chunks, lbytes;
  launch_needs(&step, 1, crit_codes != nullptr, &words, &chunks, &lbytes);
  st = ensure((void **)&c->bits, &c->bits_words, words * 8);
  if (!st) st = ensure((void **)&c->counts, &c->counts_n, chunks * (int64_t)sizeof(int));
  if (st) return st;
  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  st = enqueue_group(c, s, field, &step, 1, codes, crit, crit_codes,
                     crit_capacity, crit_count_dev, gen, true, c->bits, c->counts);
  if (st) return st;
  if (!crit_count_host) return PCRIT_OK;
  if (read_status(c, s)) return PCRIT_E_HIP;
  const int64_t count = c->h_base[1] - c->h_base[0];
  *crit_count_host = count;
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return count > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

int pcrit_classify_noalloc(pcrit_ctx *c, void *hip_stream, const float *field,
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
  set_quad(&g, quad_eligible(field, nx, g.s, g.dim));
  Step step;
  step.g = g;
  int64_t words, chunks, lbytes;
  launch_needs(&step, 1, crit_codes != nullptr, &words, &chunks, &lbytes);
  // bitmask words, then the chunk counts at a 256-byte boundary
  const int64_t counts_at = (words * 8 + 255) / 256 * 256;
  if (counts_at + chunks * (int64_t)sizeof(int) > kNoAllocScratchBytes)
    return PCRIT_E_SCRATCH;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  char *base = static_cast<char *>(noalloc_scratch(c->device));
  if (!base) return PCRIT_E_HIP;
  // Nothing in the scratch has to start at zero: the classification writes
  // every bitmask word of the level and the count kernel every chunk count
  // before they are read.  Kernel timing is not recorded here.
  const uint64_t timing = c->timing;
  c->timing = 0;
  hipStream_t s = (hipStream_t)hip_stream;
  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  st = enqueue_group(c, s, field, &step, 1, codes, crit, crit_codes, crit_capacity,
                     crit_count_dev, gen, true, reinterpret_cast<uint64_t *>(base),
                     reinterpret_cast<int *>(base + counts_at));
  c->timing = timing;
  if (st) return st;
  if (!crit_count_host) return PCRIT_OK;
  if (read_status(c, s)) return PCRIT_E_HIP;
  const int64_t count = c->h_base[1] - c->h_base[0];
  *crit_count_host = count;
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return count > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

}  // extern "C"

namespace {

// Plans and enqueues a progressive call (levels k_max .. 0) on `s`: level
// steps, their grouping into launches, scratch sizing, then the launches.
// With a callback every level completes (and is reported) on its own.
// With `count` every old vertex is tested against the previous level (its
// stored or recomputed polarity mask) and the re-classified ones counted.
int enqueue_progressive(pcrit_ctx *c, hipStream_t s, const float *field,
                        int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                        uint32_t *crit, uint8_t *crit_codes, int64_t crit_capacity,
                        bool timed, bool count, pcrit_level_cb cb, void *user,
                        int *kmax_out, int *group_end, unsigned *gen_out,
                        int64_t *publish = nullptr, bool *published = nullptr) {
  if (!c || !field || !codes || crit_capacity < 0 ||
      (crit_capacity > 0 && !crit))
    return PCRIT_E_ARG;
  if (misaligned(field, 4) || (crit && misaligned(crit, 4)))
    return PCRIT_E_ARG;
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int kmax = max_level_of(nx, ny, nz);
  *kmax_out = kmax;
  Geom geo[kMaxLevels];
  for (int k = 0; k <= kmax; k++) {
    st = make_geom(nx, ny, nz, k, &geo[k]);
    if (st) return st;
  }
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;

  // Steps in order (i = kmax - k) and their grouping into launches: the
  // leading run of small levels is fused (up to kMaxFused per launch) unless
  // a per-level callback wants each level to complete on its own.
  Step steps[kMaxLevels];
  for (int i = 0; i <= kmax; i++) {
    const int k = kmax - i;
    Step &sp = steps[i];
    sp.g = geo[k];
    sp.slot = i;
    if (i > 0 && count) {
      sp.prev = &geo[k + 1];
      sp.dirty = true;
      sp.mask_read = (i - 1) & 1;
      sp.reclass_out = &c->flags[3 + i];
    }
  }
  for (int i = 0; i <= kmax;) {
    int j = i + 1;
    if (!cb && level_vertices(steps[i].g) <= kSmallLevel)
      while (j <= kmax && j - i < kMaxFused && level_vertices(steps[j].g) <= kSmallLevel)
        j++;
    group_end[i] = j;
    // counting: the last level of a launch stores its masks for the next
    // launch; otherwise a level of its own may take the quad tiles
    if (count && j <= kmax) steps[j - 1].mask_write = (j - 1) & 1;
    if (!count && j == i + 1)
      set_quad(&steps[i].g, quad_eligible(field, nx, steps[i].g.s, steps[i].g.dim));
    i = j;
  }
  int64_t need_words = 0, need_chunks = 0, need_l = 0, need_masks = 0;
  for (int i = 0; i <= kmax; i = group_end[i]) {
    int64_t w, ch, lb;
    launch_needs(&steps[i], group_end[i] - i, crit_codes != nullptr, &w, &ch, &lb);
    need_words = std::max(need_words, w);
    need_chunks = std::max(need_chunks, ch);
    need_l = std::max(need_l, lb);
    const Step &last = steps[group_end[i] - 1];
    if (last.mask_write >= 0)
      need_masks = std::max(need_masks,
                            level_vertices(last.g) * (last.g.dim == 3 ? 2 : 1));
  }
  // Beside mode: the finest level, when it is a launch of its own, runs
  // beside the coarser ones: its classification on `s` while they
  // (classification and compaction, in order) run on the side stream, its
  // compaction once they are done, since its list follows theirs.  The
  // levels are independent unless old vertices are tested against the
  // previous level (`count`) or coarser levels store codes the finest one
  // overwrites (list codes).  Sharing the GPU with the finest level delays
  // the coarser ones, so a caller that watches levels complete (a callback
  // or level times) gets them in turn, and so does kernel timing, which
  // wants each kernel alone.  (Running the next level's classification on
  // `s` too, with its compaction on the side stream, cost more in
  // cross-stream waits than it overlapped.)
  int ilast = 0;
  for (int i = 0; i <= kmax; i = group_end[i]) ilast = i;
  const bool beside = ilast > 0 && group_end[ilast] == ilast + 1 && !count && !cb &&
                      !timed && !crit_codes && c->timing == 0;
  st = ensure((void **)&c->bits, &c->bits_words, need_words * 8);
  if (!st) st = ensure((void **)&c->counts, &c->counts_n, need_chunks * (int64_t)sizeof(int));
  if (!st) st = ensure((void **)&c->lcodes, &c->lcodes_bytes, need_l);
  if (!st && beside) {
    int64_t w, ch, lb;
    launch_needs(&steps[ilast], 1, false, &w, &ch, &lb);
    st = ensure((void **)&c->bits2, &c->bits2_words, w * 8);
    if (!st) st = ensure((void **)&c->counts2, &c->counts2_n, ch * (int64_t)sizeof(int));
  }
  if (!st && beside) st = ensure_side(c);
  if (st) return st;
  if (need_masks > c->masks_bytes) {
    hipDeviceSynchronize();
    for (int i = 0; i < 2; i++) {
      if (c->masks[i]) hipFree(c->masks[i]);
      c->masks[i] = nullptr;
    }
    c->masks_bytes = 0;
    for (int i = 0; i < 2; i++)
      if (hipMalloc(&c->masks[i], (size_t)need_masks) != hipSuccess) return PCRIT_E_OOM;
    c->masks_bytes = need_masks;
  }

  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  // Completion events only when asked for: every record is a release on the
  // stream, which costs microseconds of GPU time.  Levels of one launch
  // complete together and share the event of its last level.
  // The start event follows a short GPU wait by which the host has queued
  // the call's kernels, so launch latency stays out of the level times.
  if (timed && (launch_wait_stamp(nullptr, kTimelineLeadUs, s) != hipSuccess ||
                hipEventRecord(c->ev_start, s) != hipSuccess))
    return PCRIT_E_HIP;
  hipStream_t t = s;  // stream of the levels before the finest
  if (beside) {
    t = c->side;
    if (hipEventRecord(c->ev_fork, s) != hipSuccess ||
        hipStreamWaitEvent(t, c->ev_fork, 0) != hipSuccess)
      return PCRIT_E_HIP;
  }
  for (int i = 0; i <= kmax; i = group_end[i]) {
    const int n = group_end[i] - i;
    const bool finest = i + n > kmax;
    // the compaction of a last launch of one level publishes the offsets
    const bool pub = publish && finest && n == 1;
    hipStream_t si = beside && !finest ? t : s;
    if (beside && finest && hipEventRecord(c->ev_join, t) != hipSuccess) return PCRIT_E_HIP;
    st = enqueue_group(c, si, field, &steps[i], n, codes, crit, crit_codes, crit_capacity,
                       nullptr, gen, finest, beside && finest ? c->bits2 : c->bits,
                       beside && finest ? c->counts2 : c->counts, pub ? publish : nullptr,
                       pub ? kmax + 2 : 0, nullptr, nullptr,
                       beside && finest ? c->ev_join : nullptr);
    if (pub) *published = true;
    if (st) return st;
    if (timed && hipEventRecord(c->ev_level[i + n - 1], si) != hipSuccess)
      return PCRIT_E_HIP;
    if (cb) {
      if (read_status(c, s)) return PCRIT_E_HIP;
      cb(kmax - i, c->h_base[i + 1] - c->h_base[i], user);
    }
  }
  *gen_out = gen;
  return PCRIT_OK;
}

}  // namespace

extern "C" {

int pcrit_progressive(pcrit_ctx *c, void *hip_stream, const float *field,
                      int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                      uint32_t *crit, uint8_t *crit_codes,
                      int64_t crit_capacity, int64_t *level_offsets_host,
                      float *level_ms_host, int64_t *reclassified_host,
                      pcrit_level_cb cb, void *user) {
  hipStream_t s = (hipStream_t)hip_stream;
  int kmax = 0, group_end[kMaxLevels];
  unsigned gen = 0;
  const bool timed = level_ms_host != nullptr;
  const bool count = reclassified_host != nullptr;
  int st = enqueue_progressive(c, s, field, nx, ny, nz, codes, crit, crit_codes,
                               crit_capacity, timed, count, cb, user, &kmax, group_end,
                               &gen);
  if (st) return st;
  if (read_status(c, s)) return PCRIT_E_HIP;
  if (level_offsets_host)
    for (int i = 0; i <= kmax + 1; i++) level_offsets_host[i] = c->h_base[i];
  if (reclassified_host)
    for (int i = 0; i <= kmax; i++)
      reclassified_host[i] = i == 0 ? 0 : (int64_t)c->h_flags[3 + i];
  if (timed)
    for (int i = 0; i <= kmax; i = group_end[i]) {
      float ms = -1.f;
      if (hipEventElapsedTime(&ms, c->ev_start, c->ev_level[group_end[i] - 1]) !=
          hipSuccess)
        ms = -1.f;
      for (int j = i; j < group_end[i]; j++) level_ms_host[j] = ms;
    }
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return c->h_base[kmax + 1] > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

int pcrit_progressive_async(pcrit_ctx *c, void *hip_stream, const float *field,
                            int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                            uint32_t *crit, int64_t crit_capacity,
                            int64_t *level_offsets_dev) {
  if (!level_offsets_dev || misaligned(level_offsets_dev, 8)) return PCRIT_E_ARG;
  hipStream_t s = (hipStream_t)hip_stream;
  int kmax = 0, group_end[kMaxLevels];
  unsigned gen = 0;
  bool published = false;
  int st = enqueue_progressive(c, s, field, nx, ny, nz, codes, crit, nullptr,
                               crit_capacity, false, false, nullptr, nullptr, &kmax,
                               group_end, &gen, level_offsets_dev, &published);
  if (st) return st;
  if (published) return PCRIT_OK;
  return launch_publish_offsets(c->level_base, kmax + 2, &c->flags[0], gen,
                                level_offsets_dev, s) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
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

// ---------------------------------------------------------------------------
// Learned refinement order and the region timeline
// ---------------------------------------------------------------------------

namespace {

// Level of the learned order's features: about 64 cells along the shortest
// axis (at least level 1).
int feature_level(int64_t nx, int64_t ny, int64_t nz, int kmax) {
  const int64_t nmin = std::min(std::min(nx, ny), nz) - 1;
  int best = 1;
  double err = 1e30;
  for (int k = 1; k <= kmax; k++) {
    const double e = fabs(log2((double)nmin / (double)((int64_t)1 << k)) - 5.0);
    if (e < err) {
      err = e;
      best = k;
    }
  }
  return std::min(best, kmax);
}

float resolution_feature(int64_t nx, int64_t ny, int64_t nz, int level) {
  const int64_t nmin = std::min(std::min(nx, ny), nz) - 1;
  return (float)(log2((double)nmin / (double)((int64_t)1 << level)) / 8.0);
}

}  // namespace

extern "C" {

int pcrit_mlp_feature_level(int64_t nx, int64_t ny, int64_t nz, int *level_host) {
  if (!level_host || nz < 2) return PCRIT_E_ARG;
  const int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int kmax = max_level_of(nx, ny, nz);
  if (kmax < 1) return PCRIT_E_DIMS;
  *level_host = feature_level(nx, ny, nz, kmax);
  return PCRIT_OK;
}

int pcrit_mlp_features(pcrit_ctx *c, void *hip_stream, const float *field, int64_t nx,
                       int64_t ny, int64_t nz, int level, uint16_t *X) {
  if (!c || !field || !X || nz < 2 || level < 1) return PCRIT_E_ARG;
  Geom g;
  const int st = make_geom(nx, ny, nz, level, &g);
  if (st) return st;
  if (misaligned(X, 16)) return PCRIT_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_mlp_features(field, nx, ny, nz, (int)g.s, (int)g.mx, (int)g.my, (int)g.mz,
                             resolution_feature(nx, ny, nz, level), X,
                             (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}

int pcrit_mlp_labels(pcrit_ctx *c, void *hip_stream, const uint8_t *codes, int64_t nx,
                     int64_t ny, int64_t nz, int level, uint8_t *labels) {
  if (!c || !codes || !labels || nz < 2 || level < 1) return PCRIT_E_ARG;
  Geom g;
  const int st = make_geom(nx, ny, nz, level, &g);
  if (st) return st;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_mlp_labels(codes, nx, ny, nz, (int)g.s, (int)g.mx, (int)g.my, (int)g.mz, labels,
                           (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}

int pcrit_mlp_forward(pcrit_ctx *c, void *hip_stream, const float *params, const uint16_t *X,
                      int64_t n, float *logits) {
  if (!c || !params || n < 0 || (n > 0 && (!X || !logits)) || misaligned(X, 16))
    return PCRIT_E_ARG;
  if (n == 0) return PCRIT_OK;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_mlp_forward(params, X, n, logits, (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}

int pcrit_mlp_backward(pcrit_ctx *c, void *hip_stream, const float *params, const uint16_t *X,
                       const uint8_t *labels, int64_t n, float *grad, float *loss) {
  if (!c || !params || !grad || !loss || n < 1 || !X || !labels || misaligned(X, 16))
    return PCRIT_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_mlp_backward(params, X, labels, n, grad, loss, (hipStream_t)hip_stream) ==
                 hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}

int pcrit_mlp_adam(pcrit_ctx *c, void *hip_stream, float *params, const float *grad, float *m,
                   float *v, float lr, int step) {
  if (!c || !params || !grad || !m || !v || step < 1 || !(lr > 0.f)) return PCRIT_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_mlp_adam(params, grad, m, v, lr, step, (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}

int pcrit_region_count(int64_t nx, int64_t ny, int64_t nz, int region_edge, int *n_host) {
  if (!n_host || nz < 2 || region_edge < 32 || region_edge > (1 << 20) ||
      (region_edge & (region_edge - 1)))
    return PCRIT_E_ARG;
  const int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int64_t n = ((ny + region_edge - 1) / region_edge) * ((nz + region_edge - 1) / region_edge);
  if (n > kMaxRegions) return PCRIT_E_ARG;
  *n_host = (int)n;
  return PCRIT_OK;
}

int pcrit_progressive_timeline(pcrit_ctx *c, void *hip_stream, const float *field, int64_t nx,
                               int64_t ny, int64_t nz, uint8_t *codes, uint32_t *crit,
                               int64_t crit_capacity, int region_edge, int order_mode,
                               int32_t *rank_host, const float *mlp_params,
                               int64_t *level_offsets_host, double *level_ms_host,
                               double *region_ms_host) {
  if (!c || !field || !codes || crit_capacity < 0 || (crit_capacity > 0 && !crit) ||
      !level_offsets_host || !level_ms_host || !region_ms_host)
    return PCRIT_E_ARG;
  if (misaligned(field, 4) || (crit && misaligned(crit, 4))) return PCRIT_E_ARG;
  int nregions = 0;
  int st = pcrit_region_count(nx, ny, nz, region_edge, &nregions);
  if (st) return st;
  if (order_mode < 0 || order_mode > 2 || (order_mode == 1 && !rank_host) ||
      (order_mode == 2 && !mlp_params))
    return PCRIT_E_ARG;
  if (order_mode == 1) {  // a permutation of the regions
    std::vector<char> seen(nregions, 0);
    for (int r = 0; r < nregions; r++) {
      const int k = rank_host[r];
      if (k < 0 || k >= nregions || seen[k]) return PCRIT_E_ARG;
      seen[k] = 1;
    }
  }
  const int kmax = max_level_of(nx, ny, nz);
  Geom geo[kMaxLevels];
  for (int k = 0; k <= kmax; k++) {
    st = make_geom(nx, ny, nz, k, &geo[k]);
    if (st) return st;
  }
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  const int E = region_edge, nry = (int)((ny + E - 1) / E);

  // Groups: the leading small levels in two launches (up to 2^18 vertices,
  // then the rest up to 2^22), every other level on its own; single levels
  // with quad tiles are refined region by region.
  Step steps[kMaxLevels];
  int group_end[kMaxLevels];
  for (int i = 0; i <= kmax; i++) {
    steps[i].g = geo[kmax - i];
    steps[i].slot = i;
  }
  for (int i = 0; i <= kmax;) {
    int j = i + 1;
    const int64_t cap = level_vertices(steps[i].g) <= ((int64_t)1 << 18) ? ((int64_t)1 << 18)
                                                                          : kSmallLevel;
    if (level_vertices(steps[i].g) <= kSmallLevel)
      while (j <= kmax && j - i < kMaxFused && level_vertices(steps[j].g) <= cap) j++;
    group_end[i] = j;
    if (j == i + 1)
      set_quad(&steps[i].g, quad_eligible(field, nx, steps[i].g.s, steps[i].g.dim));
    i = j;
  }
  // Levels refined by regions and their tile plans (as the launch makes
  // them); their tile lists are built up front, on the side stream.
  struct RegionalLevel {
    int i;
    LevelDesc l;
    int64_t list_off;
  };
  std::vector<RegionalLevel> rl;
  int64_t need_words = 0, need_chunks = 0, all_tiles = 0;
  for (int i = 0; i <= kmax; i = group_end[i]) {
    int64_t w, ch, lb;
    launch_needs(&steps[i], group_end[i] - i, false, &w, &ch, &lb);
    need_words = std::max(need_words, w);
    need_chunks = std::max(need_chunks, ch);
    if (group_end[i] == i + 1 && steps[i].g.quad) {
      LevelDesc l{};
      l.mx = (int)steps[i].g.mx;
      l.my = (int)steps[i].g.my;
      l.mz = (int)steps[i].g.mz;
      plan_level_quad(l, std::min(kQuadZChunk, E / (int)steps[i].g.s));
      rl.push_back({i, l, all_tiles});
      all_tiles += l.ntiles;
    }
  }
  const int nrl = (int)rl.size();
  st = ensure((void **)&c->bits, &c->bits_words, need_words * 8);
  if (!st) st = ensure((void **)&c->counts, &c->counts_n, need_chunks * (int64_t)sizeof(int));
  if (st) return st;
  const int lf = feature_level(nx, ny, nz, kmax);
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t left_bytes = up(4 * (int64_t)kCounterStride * nregions),
                scr_bytes = up(4 * kRegionScratchInts(nregions));
  const int64_t o_stamp = 0, o_rstamp = o_stamp + up(8 * (kMaxLevels + 2)),
                o_left = o_rstamp + up(8 * (int64_t)(kmax + 1) * nregions),
                o_rank = o_left + left_bytes * std::max(nrl, 1),
                o_scr = o_rank + up(4 * (int64_t)nregions),
                o_score = o_scr + scr_bytes * std::max(nrl, 1),
                o_list = o_score + up(4 * (int64_t)kCounterStride * nregions),
                total = o_list + up(4 * std::max<int64_t>(all_tiles, 1));
  st = ensure(&c->tl, &c->tl_bytes, total);
  if (st) return st;
  char *tb = static_cast<char *>(c->tl);
  uint64_t *stamps = reinterpret_cast<uint64_t *>(tb + o_stamp);
  uint64_t *rstamps = reinterpret_cast<uint64_t *>(tb + o_rstamp);
  int *rank = reinterpret_cast<int *>(tb + o_rank);
  auto level_left = [&](int k) { return reinterpret_cast<unsigned *>(tb + o_left + k * left_bytes); };
  auto level_scr = [&](int k) { return reinterpret_cast<int *>(tb + o_scr + k * scr_bytes); };
  auto level_list = [&](int k) { return reinterpret_cast<int *>(tb + o_list) + rl[k].list_off; };
  if (order_mode != 2) {
    std::vector<int> h(nregions);
    for (int r = 0; r < nregions; r++) h[r] = order_mode == 1 ? rank_host[r] : r;
    if (hipMemcpyAsync(rank, h.data(), sizeof(int) * nregions, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PCRIT_E_HIP;
  }
  if (hipMemsetAsync(rstamps, 0, 8 * (size_t)(kmax + 1) * nregions, s) != hipSuccess)
    return PCRIT_E_HIP;

  const bool learn = order_mode == 2 && nrl > 0;
  if (nrl > 0 && ensure_side(c)) return PCRIT_E_HIP;

  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  int nstamp = 0;
  int stamp_of_group[kMaxLevels];
  // the clock starts once the host has queued the call's work: a short
  // wait on the GPU ahead of the first stamp keeps launch latency out of
  // the timeline
  if (launch_wait_stamp(&stamps[nstamp++], kTimelineLeadUs, s) != hipSuccess)
    return PCRIT_E_HIP;
  if (nrl > 0) {
    // on the side stream, overlapping the leading levels: the learned order
    // (inputs of level lf, logits, region scores, ranks), then the tile
    // lists of every region-refined level
    hipStream_t s2 = c->side;
    if (hipEventRecord(c->ev_fork, s) != hipSuccess ||
        hipStreamWaitEvent(s2, c->ev_fork, 0) != hipSuccess)
      return PCRIT_E_HIP;
    if (learn) {
      float *score = reinterpret_cast<float *>(tb + o_score);
      const Geom &gf = geo[lf];
      if (launch_mlp_region_scores(mlp_params, field, nx, ny, (int)gf.s, (int)gf.mx, (int)gf.my,
                                   (int)gf.mz, resolution_feature(nx, ny, nz, lf), E, nry,
                                   nregions, score, s2) != hipSuccess ||
          launch_region_rank(score, kCounterStride, nregions, rank, s2) != hipSuccess)
        return PCRIT_E_HIP;
    }
    for (int k = 0; k < nrl; k++)
      if (launch_region_tiles(rl[k].l, kQuadRows, (int)steps[rl[k].i].g.s, E, nry, nregions, rank,
                              level_list(k), level_left(k), level_scr(k), s2) != hipSuccess)
        return PCRIT_E_HIP;
    if (hipEventRecord(c->ev_join, s2) != hipSuccess) return PCRIT_E_HIP;
  }
  bool joined = false;
  int k_rl = 0;
  for (int i = 0; i <= kmax; i = group_end[i]) {
    const int n = group_end[i] - i;
    const bool regional = n == 1 && steps[i].g.quad;
    RegionHooks rh;
    if (regional) {
      if (!joined) {
        // the first region-refined level waits for the side stream
        if (hipStreamWaitEvent(s, c->ev_join, 0) != hipSuccess) return PCRIT_E_HIP;
        joined = true;
      }
      rh.E = E;
      rh.nry = nry;
      rh.nregions = nregions;
      rh.rank = rank;
      rh.tile_list = level_list(k_rl);
      rh.scratch = level_scr(k_rl);
      rh.left = level_left(k_rl);
      rh.stamp = rstamps + (int64_t)i * nregions;
      rh.prebuilt = true;
      k_rl++;
    }
    st = enqueue_group(c, s, field, &steps[i], n, codes, crit, nullptr, crit_capacity, nullptr,
                       gen, i + n > kmax, c->bits, c->counts, nullptr, 0,
                       regional ? &rh : nullptr);
    if (st) return st;
    stamp_of_group[i] = nstamp;
    if (launch_stamp(&stamps[nstamp++], s) != hipSuccess) return PCRIT_E_HIP;
  }
  std::vector<uint64_t> hs(nstamp), hr((size_t)(kmax + 1) * nregions);
  if (order_mode == 2 && rank_host) {
    if (!learn) {
      for (int r = 0; r < nregions; r++) rank_host[r] = r;
    } else if (hipMemcpyAsync(rank_host, rank, sizeof(int) * nregions, hipMemcpyDeviceToHost,
                              s) != hipSuccess) {
      return PCRIT_E_HIP;
    }
  }
  if (hipMemcpyAsync(hs.data(), stamps, 8 * (size_t)nstamp, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hr.data(), rstamps, 8 * hr.size(), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      read_status(c, s))
    return PCRIT_E_HIP;
  // GPU clock: 100 MHz
  auto ms = [&](uint64_t t) { return (double)(int64_t)(t - hs[0]) * 1e-5; };
  for (int i = 0; i <= kmax; i = group_end[i]) {
    const double done = ms(hs[stamp_of_group[i]]);
    const bool regional = group_end[i] == i + 1 && steps[i].g.quad;
    for (int j = i; j < group_end[i]; j++) {
      level_ms_host[j] = done;
      for (int r = 0; r < nregions; r++) {
        const uint64_t t = hr[(size_t)j * nregions + r];
        region_ms_host[(size_t)j * nregions + r] = regional && t ? ms(t) : done;
      }
    }
  }
  for (int i = 0; i <= kmax + 1; i++) level_offsets_host[i] = c->h_base[i];
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return c->h_base[kmax + 1] > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}


// ------------------------------------------------------------------------
// Batches of independent fields (level 0): groups of up to kMaxFused fields
// share one classification and one compaction launch; every field keeps its
// own pointers and sizes, and the lists land in field order.
int pcrit_classify_batch(pcrit_ctx *c, void *hip_stream, int n_fields,
                         const pcrit_batch_field *fields_host, uint32_t *crit,
                         uint8_t *crit_codes, int64_t crit_capacity, int64_t *offsets_host,
                         int64_t *offsets_dev) {
  if (!c || n_fields < 1 || n_fields > PCRIT_MAX_BATCH_FIELDS || !fields_host || crit_capacity < 0 ||
      (crit_capacity > 0 && !crit) || (crit && misaligned(crit, 4)) ||
      (offsets_dev && misaligned(offsets_dev, 8)))
    return PCRIT_E_ARG;
  std::vector<Step> steps((size_t)n_fields);
  int dim = 0;
  int64_t words = 0, chunks = 0;
  for (int i = 0; i < n_fields; i++) {
    const pcrit_batch_field &fd = fields_host[i];
    if (!fd.field || !fd.codes || misaligned(fd.field, 4)) return PCRIT_E_ARG;
    Geom g;
    const int st = make_geom(fd.nx, fd.ny, fd.nz, 0, &g);
    if (st) return st;
    if (dim == 0) dim = g.dim;
    if (g.dim != dim) return PCRIT_E_ARG;  // one triangulation per call
    Step &sp = steps[(size_t)i];
    sp.g = g;
    sp.f = fd.field;
    sp.codes = fd.codes;
    sp.batch = true;
    sp.want = c->batch_want;
    sp.slot = i;
  }
  const int G = c->batch_group;
  // scratch for the largest group
  for (int i0 = 0; i0 < n_fields; i0 += G) {
    const int n = std::min(G, n_fields - i0);
    int64_t w, ch, lb;
    launch_needs(&steps[(size_t)i0], n, false, &w, &ch, &lb);
    words = std::max(words, w);
    chunks = std::max(chunks, ch);
  }
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  // More than one group: group g+1 is classified on hip_stream while group
  // g is compacted on the side stream (compactions in order there, so the
  // lists still land in field order), each group on scratch set g % 2.
  const int ngroups = (n_fields + G - 1) / G;
  const bool piped = ngroups > 1;
  int st = ensure((void **)&c->bits, &c->bits_words, words * 8);
  if (!st) st = ensure((void **)&c->counts, &c->counts_n, chunks * (int64_t)sizeof(int));
  if (!st && piped) st = ensure((void **)&c->bits2, &c->bits2_words, words * 8);
  if (!st && piped) st = ensure((void **)&c->counts2, &c->counts2_n, chunks * (int64_t)sizeof(int));
  if (!st && piped) st = ensure_side(c);
  int64_t *off = offsets_dev;
  if (!st && !off) {
    st = ensure((void **)&c->boff, &c->boff_bytes, 8 * (int64_t)(n_fields + 1));
    off = c->boff;
  }
  if (st) return st;
  // the first group's lists start at off[0] = 0 (a kernel, not a memset, so
  // that the call can be captured in a graph)
  if (launch_zero_i64(off, 1, s) != hipSuccess) return PCRIT_E_HIP;
  const unsigned gen = next_gen(c);
  reset_kernel_marks(c);
  for (int i0 = 0, g = 0; i0 < n_fields; i0 += G, g++) {
    const int n = std::min(G, n_fields - i0);
    const int k = g & 1;
    // set k is free once group g-2's compaction is done
    if (piped && g >= 2 && hipStreamWaitEvent(s, c->ev_cmp[k], 0) != hipSuccess)
      return PCRIT_E_HIP;
    st = enqueue_group(c, s, steps[(size_t)i0].f, &steps[(size_t)i0], n, steps[(size_t)i0].codes,
                       crit, crit_codes, crit_capacity, nullptr, gen, true,
                       k ? c->bits2 : c->bits, k ? c->counts2 : c->counts, nullptr, 0, nullptr,
                       off, nullptr, piped ? c->side : nullptr, piped ? c->ev_cls[k] : nullptr);
    if (st) return st;
    if (piped && hipEventRecord(c->ev_cmp[k], c->side) != hipSuccess) return PCRIT_E_HIP;
  }
  if (piped && (hipEventRecord(c->ev_join, c->side) != hipSuccess ||
                hipStreamWaitEvent(s, c->ev_join, 0) != hipSuccess))
    return PCRIT_E_HIP;
  if (!offsets_host) return PCRIT_OK;
  if (hipMemcpyAsync(offsets_host, off, 8 * (size_t)(n_fields + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      read_status(c, s))
    return PCRIT_E_HIP;
  if (c->h_flags[0] == gen) return PCRIT_E_NAN;
  return offsets_host[n_fields] > crit_capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

// ------------------------------------------------------------------------
// Batch launch configuration and its autotuner.
int pcrit_set_batch_config(pcrit_ctx *c, int group, int64_t want_tiles) {
  if (!c || group < 0 || group > PCRIT_BATCH_GROUP_MAX || want_tiles < 0 ||
      (want_tiles > 0 && (want_tiles < kBatchWantMin || want_tiles > kBatchWantMax)))
    return PCRIT_E_ARG;
  c->batch_group = group ? group : kBatchGroupDefault;
  c->batch_want = want_tiles ? want_tiles : kBatchWantDefault;
  return PCRIT_OK;
}

int pcrit_get_batch_config(pcrit_ctx *c, int *group, int64_t *want_tiles) {
  if (!c || !group || !want_tiles) return PCRIT_E_ARG;
  *group = c->batch_group;
  *want_tiles = c->batch_want;
  return PCRIT_OK;
}

int pcrit_batch_autotune(pcrit_ctx *c, void *hip_stream, int n_fields,
                         const pcrit_batch_field *fields_host, uint32_t *crit,
                         uint8_t *crit_codes, int64_t crit_capacity, int reps,
                         double *times_ms_host, int *group_out, int64_t *want_out) {
  static const int kGroups[] = {8, 16};
  static const int64_t kWants[] = {128, 256, 512, 1024, 2048, 4096};
  static_assert(sizeof(kGroups) / sizeof(kGroups[0]) * sizeof(kWants) / sizeof(kWants[0]) ==
                    PCRIT_BATCH_TUNE_CANDIDATES,
                "candidate count");
  if (!c || reps < 1 || reps > 100) return PCRIT_E_ARG;
  const int g0 = c->batch_group;
  const int64_t w0 = c->batch_want;
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int64_t> off((size_t)std::max(n_fields, 0) + 1);
  // one checked call first: arguments, capacity and NaN, with the current
  // configuration
  int st = pcrit_classify_batch(c, hip_stream, n_fields, fields_host, crit, crit_codes,
                                crit_capacity, off.data(), nullptr);
  if (st) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return PCRIT_E_HIP;
  }
  double best = -1.0;
  int bg = g0;
  int64_t bw = w0;
  int k = 0;
  for (int gi : kGroups)
    for (int64_t wi : kWants) {
      c->batch_group = gi;
      c->batch_want = wi;
      // an untimed call grows the scratch this configuration needs
      st = pcrit_classify_batch(c, hip_stream, n_fields, fields_host, crit, crit_codes,
                                crit_capacity, nullptr, nullptr);
      if (!st && hipEventRecord(e0, s) != hipSuccess) st = PCRIT_E_HIP;
      for (int r = 0; r < reps && !st; r++)
        st = pcrit_classify_batch(c, hip_stream, n_fields, fields_host, crit, crit_codes,
                                  crit_capacity, nullptr, nullptr);
      float ms = 0.f;
      if (!st && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = PCRIT_E_HIP;
      if (st) break;
      const double per = (double)ms / reps;
      if (times_ms_host) times_ms_host[k] = per;
      if (best < 0 || per < best) {
        best = per;
        bg = gi;
        bw = wi;
      }
      k++;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) {
    c->batch_group = g0;
    c->batch_want = w0;
    return st;
  }
  c->batch_group = bg;
  c->batch_want = bw;
  if (group_out) *group_out = bg;
  if (want_out) *want_out = bw;
  // leave the caller's buffers holding the batch's result (the same under
  // every configuration)
  return pcrit_classify_batch(c, hip_stream, n_fields, fields_host, crit, crit_codes,
                              crit_capacity, off.data(), nullptr);
}

// ------------------------------------------------------------------------
// Order field and extremum lists.
int pcrit_order_field(pcrit_ctx *c, void *hip_stream, const float *field, int64_t nx,
                      int64_t ny, int64_t nz, uint32_t *rank, uint32_t *sorted) {
  if (!c || !field || !rank || !sorted || misaligned(field, 4) || misaligned(rank, 4) ||
      misaligned(sorted, 4))
    return PCRIT_E_ARG;
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int64_t n = nx * ny * nz;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  st = ensure(&c->ord, &c->ord_bytes, order_scratch_bytes(n));
  if (st) return st;
  const unsigned gen = next_gen(c);
  if (launch_order_field(field, n, rank, sorted, c->ord, &c->flags[0], gen, s) != hipSuccess ||
      read_status(c, s))
    return PCRIT_E_HIP;
  return c->h_flags[0] == gen ? PCRIT_E_NAN : PCRIT_OK;
}

int pcrit_extrema(pcrit_ctx *c, void *hip_stream, const uint8_t *codes, int64_t nx, int64_t ny,
                  int64_t nz, uint32_t *out, int64_t capacity, int64_t *counts_host) {
  if (!c || !codes || capacity < 0 || (capacity > 0 && !out) || !counts_host ||
      (out && misaligned(out, 4)))
    return PCRIT_E_ARG;
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  const int64_t rows = ny * nz, rowwords = (nx + 63) / 64, words = rows * rowwords;
  const bool small = small_chunks(2 * words);
  const int64_t cw = small ? kSmallChunkWords : kChunkWords;
  const int64_t chunks_per = (words + cw - 1) / cw;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  st = ensure((void **)&c->bits, &c->bits_words, 2 * words * 8);
  if (!st) st = ensure((void **)&c->counts, &c->counts_n, 2 * chunks_per * (int64_t)sizeof(int));
  if (!st) st = ensure((void **)&c->boff, &c->boff_bytes, 8 * 3);
  if (st) return st;
  CompactArgs b{};
  b.nl = 2;
  b.nchunks = (int)(2 * chunks_per);
  for (int l = 0; l < 2; l++) {
    CompactLevel &q = b.lv[l];
    q.codes = codes;
    q.nx = nx;
    q.ny = ny;
    q.bits = c->bits + l * words;
    q.words = words;
    q.rowwords = (int)rowwords;
    q.mx = (int)nx;
    q.my = (int)ny;
    q.s = 1;
    q.slot = l;
    q.chunk_begin = (int)(l * chunks_per);
    q.linear = nx == rowwords * 64;
  }
  b.crit = out;
  b.cap = capacity;
  b.level_base = c->boff;
  b.nan_flag = &c->flags[0];
  b.gen = next_gen(c);
  b.counts = c->counts;
  b.reclass_acc = c->reclass_acc;
  int64_t off[3];
  if (launch_zero_i64(c->boff, 1, s) != hipSuccess ||
      launch_extrema_bits(codes, nx, rows, (int)rowwords, c->bits, s) != hipSuccess ||
      launch_compact(b, small, s) != hipSuccess ||
      hipMemcpyAsync(off, c->boff, sizeof(off), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PCRIT_E_HIP;
  counts_host[0] = off[1] - off[0];
  counts_host[1] = off[2] - off[1];
  return off[2] > capacity ? PCRIT_E_CAPACITY : PCRIT_OK;
}

int pcrit_lts_propagate(pcrit_ctx *c, void *hip_stream, const float *field,
                        const uint32_t *rank, int64_t nx, int64_t ny, int64_t nz,
                        const uint32_t *extrema, int64_t n_extrema, int maxima, float epsilon,
                        int max_visited, int max_frontier, uint8_t *status, int32_t *saddle,
                        uint16_t *visited) {
  static_assert(PCRIT_LTS_MAX_VISITED == kLtsMaxVisited && PCRIT_LTS_MAX_FRONTIER == kLtsMaxFrontier,
                "budget limits");
  if (!c || !field || !rank || n_extrema < 0 ||
      (n_extrema > 0 && (!extrema || !status || !saddle || !visited)) ||
      misaligned(field, 4) || misaligned(rank, 4) || (extrema && misaligned(extrema, 4)) ||
      (saddle && misaligned(saddle, 4)) || (visited && misaligned(visited, 2)) ||
      epsilon != epsilon || max_visited < 2 || max_visited > PCRIT_LTS_MAX_VISITED ||
      max_frontier < 14 || max_frontier > PCRIT_LTS_MAX_FRONTIER)
    return PCRIT_E_ARG;
  const int st = check_dims(nx, ny, nz);
  if (st) return st;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  return launch_lts_propagate(field, rank, nx, ny, nz, extrema, n_extrema, maxima != 0, epsilon,
                              max_visited, max_frontier, status, saddle, visited,
                              (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}
int pcrit_lts_merged(pcrit_ctx *c, void *hip_stream, const float *field, const uint32_t *rank,
                     int64_t nx, int64_t ny, int64_t nz, const uint32_t *extrema,
                     int64_t n_extrema, int maxima, float epsilon, int max_visited,
                     int max_frontier, uint8_t *status, int32_t *saddle, uint16_t *visited) {
  if (!c || !field || !rank || n_extrema < 0 || n_extrema > kLtsMaxMerged ||
      (n_extrema > 0 && (!extrema || !status || !saddle || !visited)) ||
      misaligned(field, 4) || misaligned(rank, 4) || (extrema && misaligned(extrema, 4)) ||
      (saddle && misaligned(saddle, 4)) || (visited && misaligned(visited, 2)) ||
      epsilon != epsilon || max_visited < 2 || max_visited > PCRIT_LTS_MAX_VISITED ||
      max_frontier < 14 || max_frontier > PCRIT_LTS_MAX_FRONTIER)
    return PCRIT_E_ARG;
  int st = check_dims(nx, ny, nz);
  if (st) return st;
  if (n_extrema == 0) return PCRIT_OK;
  if (hipSetDevice(c->device) != hipSuccess) return PCRIT_E_HIP;
  st = ensure(&c->lts, &c->lts_bytes, (int64_t)lts_merged_scratch_bytes(n_extrema));
  if (st) return st;
  return launch_lts_merged(field, rank, nx, ny, nz, extrema, n_extrema, maxima != 0, epsilon,
                           max_visited, max_frontier, status, saddle, visited, c->lts,
                           (hipStream_t)hip_stream) == hipSuccess
             ? PCRIT_OK
             : PCRIT_E_HIP;
}
}  // extern "C"
