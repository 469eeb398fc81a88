/*
 * pcrit.h -- C ABI of the MI355X (gfx950) critical-point classifier.
 *
 * Classifies every vertex of a piecewise-linear scalar field sampled on a
 * regular grid as regular or critical, following the lower/upper-link
 * characterisation of Section 3.1 of Lukasczyk et al., "Localized
 * Topological Simplification of Scalar Data": a vertex is regular iff its
 * lower link and its upper link are both non-empty and simply connected; a
 * minimum has an empty lower link, a maximum an empty upper link, all other
 * critical vertices are saddles, degenerate when a link part has more than
 * two components.  Equal values are ordered by memory position (the order
 * field of Section 4.1): vertex u comes before v iff f(u) < f(v), or
 * f(u) == f(v) (IEEE-754 equality, so -0 == +0) and idx(u) < idx(v), with
 * idx = x + nx*(y + ny*z) the full-resolution linear index.
 *
 * Domain triangulation (the paper only asks for a PL manifold): each grid
 * cube [c, c+1]^3 is cut into the six tetrahedra c -> c+e_a -> c+e_a+e_b ->
 * c+(1,1,1), one per axis permutation, so every interior vertex has the 14
 * neighbours +-{(1,0,0),(0,1,0),(0,0,1),(1,1,0),(1,0,1),(0,1,1),(1,1,1)};
 * a 2D square is cut along its (1,1) diagonal (6 neighbours).  Level k of
 * the hierarchy is the sub-grid of samples whose coordinates are all
 * multiples of s = 2^k (n_k = (n-1)/s + 1 samples per axis), triangulated the
 * same way at stride s; going from level k+1 to level k inserts the midpoint
 * of every level-(k+1) edge.
 *
 * Conventions for every function below:
 *   - a pointer named *_host is host memory; every other data pointer is
 *     device memory on the context's device;
 *   - the field is float32, C order [z][y][x] (x fastest), nx*ny*nz
 *     samples; nz == 1 selects the 2D triangulation;
 *   - every active axis needs >= 2 samples and nx*ny*nz <= 2^32 - 1; a
 *     plane must hold at most 2^30 - 1 samples (nx*ny in 3D, nx in 2D):
 *     the kernels address it through buffer descriptors whose byte range
 *     ends at 2^32 - 1;
 *   - the caller owns and frees every buffer it passes in; the context owns
 *     only its lookup tables, scratch and events;
 *   - a call returns PCRIT_OK or a negative status; argument errors are
 *     detected before anything is enqueued and write nothing;
 *   - work is enqueued on `hip_stream` (a hipStream_t; NULL = the default
 *     stream); a context serves one stream at a time and is not thread-safe.
 *
 * Code byte per classified vertex (written into the full-resolution `codes`
 * array at the vertex's position; other positions are left untouched):
 *   bits 0-2  number of connected components of the lower link (0..6)
 *   bits 3-5  number of connected components of the upper link (0..6)
 *   bit  6    the vertex lies on the boundary of its level grid
 *   bit  7    boundary vertex whose lower or upper link is connected but not
 *             simply connected (it has a 1-cycle)
 * A vertex is critical iff NOT (lower == 1 and upper == 1 and bit 7 == 0).
 * Type: lower == 0 minimum; upper == 0 maximum; otherwise a saddle with
 * multiplicities lower-1 (index-1 part) and upper-1 (index-(d-1) part).
 */
#ifndef PCRIT_H
#define PCRIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCRIT_OK 0
#define PCRIT_E_ARG (-1)      /* NULL/misaligned pointer, bad argument */
#define PCRIT_E_DIMS (-2)     /* an active axis < 2 samples, N >= 2^32, or a
                                 plane of 2^30 samples or more */
#define PCRIT_E_LEVEL (-3)    /* 2^level > n-1 on some active axis */
#define PCRIT_E_CAPACITY (-4) /* critical list larger than its capacity */
#define PCRIT_E_NAN (-5)      /* a sample of the level is NaN */
#define PCRIT_E_HIP (-6)      /* a HIP runtime call failed */
#define PCRIT_E_OOM (-7)      /* device allocation of scratch failed */
#define PCRIT_E_SCRATCH (-8)  /* level too large for the fixed scratch of
                                 pcrit_classify_noalloc */

/* Size in bytes of the fixed per-GPU scratch of pcrit_classify_noalloc. */
#define PCRIT_NOALLOC_SCRATCH_BYTES (32ll << 20)

typedef struct pcrit_ctx pcrit_ctx;

/* Create a context on HIP device `hip_device`: uploads the link lookup
 * tables (16 KiB + 64 B).  *out receives the context, or NULL on error. */
int pcrit_create(pcrit_ctx **out, int hip_device);

/* Release the context's device memory and events (NULL is a no-op).  Work
 * still enqueued that uses the context must have completed. */
void pcrit_destroy(pcrit_ctx *ctx);

/* Static description of a status code. */
const char *pcrit_strerror(int status);

/* Host-only.  Coarsest level of the hierarchy: the largest k with
 * 2^k <= n-1 on every active axis. */
int pcrit_max_level(int64_t nx, int64_t ny, int64_t nz, int *k_max_host);

/* Host-only.  Samples per axis of level `level`: m3_host[0..2] = n_x, n_y,
 * n_z of the level (n_z = 1 in 2D). */
int pcrit_level_dims(int64_t nx, int64_t ny, int64_t nz, int level,
                     int64_t *m3_host);

/* Host-only.  The link-pattern table the kernels use: for every polarity
 * mask m over the neighbours (bit j = 1 iff neighbour j comes after the
 * vertex in the order) the entry is c0 | c1 << 3, where c0 (c1) is the
 * number of connected components of the link vertices whose bit is 0 (1)
 * in the link graph (two neighbours of a vertex are joined iff their offset
 * difference is itself a neighbour offset).  dim = 3: 16384 entries over the
 * 14 offsets in the order
 *   (0,0,-1) (-1,0,-1) (0,-1,-1) (-1,-1,-1)
 *   (-1,0,0) (1,0,0) (0,-1,0) (0,1,0) (-1,-1,0) (1,1,0)
 *   (0,0,1) (1,0,1) (0,1,1) (1,1,1)              as (dx,dy,dz);
 * dim = 2: 64 entries over (-1,0) (1,0) (0,-1) (0,1) (-1,-1) (1,1).
 * `size` must be at least the entry count.  Ownership stays with the
 * caller. */
int pcrit_link_table(int dim, uint8_t *table_host, int64_t size);

/* Classify every vertex of level `level` (direct, one pass).
 *   field            device, nx*ny*nz float32 (4-byte aligned)
 *   codes            device, nx*ny*nz bytes; the code of each level vertex
 *                    is written at its full-resolution position
 *   crit             device, ascending full-resolution indices (uint32) of
 *                    the critical level vertices, at most crit_capacity
 *   crit_codes       device or NULL; if set, crit_codes[i] = code of crit[i]
 *   crit_count_host  host or NULL; if set the call synchronises the stream
 *                    and stores the number of critical vertices (also when
 *                    it exceeds crit_capacity: then PCRIT_E_CAPACITY is
 *                    returned and only the first crit_capacity entries are
 *                    written; codes are complete)
 *   crit_count_dev   device int64 or NULL; if set, the count is written
 *                    there asynchronously (no synchronisation); it is set to
 *                    -1 if a NaN was found.
 * With crit_count_host == NULL the call does not synchronise, and
 * PCRIT_E_NAN / PCRIT_E_CAPACITY can only be observed through
 * crit_count_dev.  The result does not depend on the launch configuration:
 * it is the unique classification defined above. */
int pcrit_classify(pcrit_ctx *ctx, void *hip_stream, const float *field,
                   int64_t nx, int64_t ny, int64_t nz, int level,
                   uint8_t *codes, uint32_t *crit, uint8_t *crit_codes,
                   int64_t crit_capacity, int64_t *crit_count_host,
                   int64_t *crit_count_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * classification as pcrit_classify, with the same arguments, results and
 * errors, but the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  Its scratch (the level's critical bitmask,
 * one 64-bit word per 64 columns of each level row, then 4 bytes per
 * compaction chunk) lives in a fixed device array of
 * PCRIT_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; its
 * device address is looked up by pcrit_create.  A level whose scratch does
 * not fit (about 2^28 vertices with rows of a multiple of 64 columns) is
 * rejected with PCRIT_E_SCRATCH before anything is enqueued.  Every call on
 * one GPU shares that GPU's array, whatever its context or stream: calls
 * that overlap in time on one GPU race and must be serialised by the
 * caller.  Nothing in the array needs clearing between calls (every word a
 * call reads, it has written first).  Kernel timing
 * (pcrit_set_kernel_timing) is not recorded by this call. */
int pcrit_classify_noalloc(pcrit_ctx *ctx, void *hip_stream, const float *field,
                           int64_t nx, int64_t ny, int64_t nz, int level,
                           uint8_t *codes, uint32_t *crit, uint8_t *crit_codes,
                           int64_t crit_capacity, int64_t *crit_count_host,
                           int64_t *crit_count_dev);

/* Called after a level of pcrit_progressive completed (the stream is
 * synchronised first): level, number of critical vertices of that level. */
typedef void (*pcrit_level_cb)(int level, int64_t count, void *user);

/* Progressive classification: levels k_max, k_max-1, ..., 0 in turn, each
 * level's list complete before the next level's list is written.  When the
 * caller does not watch the levels complete (no callback, no level times)
 * and asks for no re-classification count or list codes, and kernel timing
 * is off, the finest level's classification runs beside the coarser levels,
 * which then run on the context's second stream (forked from and joined
 * back to hip_stream by events; the call's work still ends on hip_stream):
 * the call ends sooner, its coarser levels complete later.
 * A vertex already
 * present at level k+1 needs re-classifying at level k only if its polarity
 * mask or its set of absent (off-grid) neighbours changed, i.e. if some new
 * neighbour (the midpoint of its level-(k+1) edge) lies on the other side of
 * it than that edge's far end; otherwise its code and critical status are
 * unchanged, because the code is a function of the mask and the absent set
 * only.  The kernels classify every vertex of every level (an old vertex's
 * code read again equals the kept one, and its row is classified anyway
 * for the new vertices around it); on request they also count the old
 * vertices that changed (reclassified_host).
 *   codes         device, nx*ny*nz bytes; ends holding the level-0 code of
 *                 every vertex (stored by the level-0 pass; coarser levels
 *                 store theirs there only when crit_codes is set)
 *   crit          device; the ascending critical list of each level,
 *                 concatenated coarse to fine; crit_capacity entries
 *                 (the sum of the level sizes is always enough)
 *   crit_codes    device or NULL, as for pcrit_classify
 *   level_offsets_host  host, k_max+2 entries or NULL: the list of level k
 *                 is crit[off[i] .. off[i+1]) with i = k_max - k
 *   level_ms_host host, k_max+1 entries or NULL: milliseconds from the start
 *                 of the call's first kernel to the completion of level k,
 *                 at index i = k_max - k (stream-event timing; NULL records
 *                 no events).  The start event follows a 0.3 ms wait on the
 *                 GPU by which the host has queued the call's kernels, so
 *                 host launch latency stays out.  Levels whose work shares
 *                 one launch (see below) report the same time
 *   reclassified_host  host, k_max+1 entries or NULL: number of old vertices
 *                 whose polarity mask or absent set changed at each level
 *                 (index i; 0 for level k_max).  Non-NULL makes the call
 *                 test every old vertex against the previous level's
 *                 polarity masks (stored between launches), which costs
 *                 memory traffic; NULL skips the test
 *   cb, user      optional per-level callback (forces a synchronisation per
 *                 level)
 * Levels of at most 2^22 vertices are latency bound: unless cb is set, the
 * leading run of such levels (up to 16) is classified in one launch and
 * compacted in one more; their old vertices are then tested against the
 * previous level's masks recomputed from the field, with the same result.
 * The call always synchronises the stream at its end.  Returns
 * PCRIT_E_CAPACITY (offsets still report the required sizes) or
 * PCRIT_E_NAN as pcrit_classify does. */
int pcrit_progressive(pcrit_ctx *ctx, void *hip_stream, const float *field,
                      int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                      uint32_t *crit, uint8_t *crit_codes,
                      int64_t crit_capacity, int64_t *level_offsets_host,
                      float *level_ms_host, int64_t *reclassified_host,
                      pcrit_level_cb cb, void *user);

/* The same progressive classification, enqueued without any host
 * synchronisation (for pipelines that issue one call after another on a
 * stream and look at the results later): no list codes, timing or callback.
 *   level_offsets_dev  device, k_max+2 int64 (8-byte aligned): written
 *                 asynchronously when the call's work completes, as
 *                 level_offsets_host of pcrit_progressive; the last entry is
 *                 -1 if a NaN sample was found.  An entry above
 *                 crit_capacity means the lists did not fit (only the first
 *                 crit_capacity entries are written).
 * Returns PCRIT_OK once the work is enqueued, or an argument / HIP error
 * (nothing enqueued).  Calls on one context must share one stream. */
int pcrit_progressive_async(pcrit_ctx *ctx, void *hip_stream, const float *field,
                            int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                            uint32_t *crit, int64_t crit_capacity,
                            int64_t *level_offsets_dev);

/* Measurement.  Every later call records a HIP event pair on its stream
 * around the classification kernel and around the compaction kernels of
 * each level k whose bit k is set in level_mask (0 disables; the records
 * add a few microseconds of stream time each).  pcrit_kernel_ms then
 * returns, for the most recent call, the durations in milliseconds of the
 * classification and of the compaction of each level (index = level, up to
 * max_levels entries each; -1 where nothing was timed).  Levels that share a
 * launch are timed as one, under the finest of them (the others read -1).
 * It synchronises on the last recorded event. */
int pcrit_set_kernel_timing(pcrit_ctx *ctx, uint64_t level_mask);
int pcrit_kernel_ms(pcrit_ctx *ctx, float *classify_ms_host,
                    float *compact_ms_host, int max_levels);

/* Host-only metric: preview quality of a coarse level's critical list
 * against the exact (level-0) list.  A preview point p (level `level`) and
 * an exact point e match when they have the same type (minimum, maximum or
 * saddle, from their codes) and the L-infinity distance of their grid
 * coordinates is at most 2^level.  Pairs are taken greedily in increasing
 * distance, then increasing preview index, then increasing exact index,
 * each point used at most once.  Returns F1 = 2*matches / (|P| + |E|)
 * (1 if both lists are empty) through *f1_host, and the match count through
 * *matches_host (may be NULL).  All pointers are host memory. */
int pcrit_preview_f1(int64_t nx, int64_t ny, int64_t nz, int level,
                     const uint32_t *preview_host,
                     const uint8_t *preview_codes_host, int64_t n_preview,
                     const uint32_t *exact_host,
                     const uint8_t *exact_codes_host, int64_t n_exact,
                     double *f1_host, int64_t *matches_host);

/* Host-only metric: as pcrit_preview_f1, but each preview point i carries
 * its own level preview_levels_host[i] (match distance 2^level), for
 * previews that mix levels (regions refined to different depths). */
int pcrit_preview_f1_levels(int64_t nx, int64_t ny, int64_t nz,
                            const uint32_t *preview_host,
                            const uint8_t *preview_codes_host,
                            const uint8_t *preview_levels_host, int64_t n_preview,
                            const uint32_t *exact_host,
                            const uint8_t *exact_codes_host, int64_t n_exact,
                            double *f1_host, int64_t *matches_host);

/* ------------------------------------------------------------------------
 * Region timeline and learned refinement order (3D grids).
 *
 * The paper classifies every vertex; it has no hierarchy and no refinement
 * order.  Here the progressive call can refine its full-resolution and
 * stride-2 levels region by region: a region is a block of region_edge
 * full-resolution rows by region_edge planes (all columns), numbered
 * rz * nry + ry with nry = ceil(ny / region_edge), and a preview at time t
 * shows each region at the finest level whose pass over that region has
 * finished.  The order only changes when a region's previews appear; every
 * vertex of every level is classified either way, so the lists and codes
 * are those of pcrit_progressive.
 *
 * A small network can choose the order: inputs are the 27 samples around a
 * vertex of a coarse level (the 3x3x3 neighbourhood at that level's stride,
 * z slowest, x fastest, minus the centre sample, divided by the largest
 * magnitude among them, 0 if all are equal), then log2((n_min - 1) / 2^level)
 * / 8 with n_min the shortest axis, then 4 zeros: 32 BF16 values per vertex
 * (uint16 bit patterns).  The network is 32 -> 64 -> 64 -> 1: h1 = GELU(x W1
 * + b1), h2 = GELU(h1 W2 + b2), logit = h2 . w3 + b3, GELU(u) = u/2 (1 +
 * erf(u / sqrt 2)) (the kernels evaluate erf to within 1.5e-7, Abramowitz
 * and Stegun 7.1.26).  Parameters: PCRIT_MLP_PARAMS floats, FP32, in the
 * order W1 [32][64] (input-major), b1 [64], W2 [64][64], b2 [64], w3 [64],
 * b3.  The kernels round W1, W2 and w3 to BF16 (nearest even), x and h1 are
 * BF16, products accumulate in FP32; b1, b2, b3, h2 and the output are FP32.
 * Its training target for a vertex v of level k (stride s) is the fraction
 * of critical vertices (level-0 codes) among the full-resolution vertices
 * within [v - s/2, v + s/2) on every axis (clipped to the grid), stored as
 * the byte ceil(255 * count / volume) and read as byte / 255.  A region's
 * score is the sum of the sigmoid of its vertices' logits (an estimate of
 * its number of exact critical points over the cell volume); regions are
 * refined by decreasing score.
 * ---------------------------------------------------------------------- */
#define PCRIT_MLP_PARAMS 6337
#define PCRIT_MLP_INPUTS 32

/* Host-only.  Coarse level whose vertices the learned order scores (about
 * 64 cells along the shortest axis, at least 1).  3D only. */
int pcrit_mlp_feature_level(int64_t nx, int64_t ny, int64_t nz, int *level_host);

/* Network inputs of every vertex of level `level` (>= 1, 3D): X is device
 * memory, 16-byte aligned, n_level x 32 uint16 (BF16), level-local C order. */
int pcrit_mlp_features(pcrit_ctx *ctx, void *hip_stream, const float *field,
                       int64_t nx, int64_t ny, int64_t nz, int level, uint16_t *X);

/* Training targets of the vertices of level `level` from full-resolution
 * level-0 codes (device): labels[i] = ceil(255 * critical fraction of the
 * cell) (device, n_level bytes). */
int pcrit_mlp_labels(pcrit_ctx *ctx, void *hip_stream, const uint8_t *codes,
                     int64_t nx, int64_t ny, int64_t nz, int level, uint8_t *labels);

/* logits[i] of the n inputs X (all device memory). */
int pcrit_mlp_forward(pcrit_ctx *ctx, void *hip_stream, const float *params,
                      const uint16_t *X, int64_t n, float *logits);

/* Gradient of the mean binary cross-entropy of the logits of X against
 * the targets labels / 255 with respect to params: written to grad (PCRIT_MLP_PARAMS
 * floats, overwritten); *loss (device float) receives the sum of the
 * per-sample losses.  The weight-gradient products run on the matrix cores
 * with BF16 operands (the back-propagated signals and the activations
 * rounded to BF16, FP32 accumulation), so the gradient is the exact one of
 * the forward pass above to about 1 %.  All pointers are device memory;
 * n >= 1. */
int pcrit_mlp_backward(pcrit_ctx *ctx, void *hip_stream, const float *params,
                       const uint16_t *X, const uint8_t *labels, int64_t n,
                       float *grad, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
 * number step >= 1) on params with moments m and v (device, each
 * PCRIT_MLP_PARAMS floats, m and v zero before the first step). */
int pcrit_mlp_adam(pcrit_ctx *ctx, void *hip_stream, float *params,
                   const float *grad, float *m, float *v, float lr, int step);

/* Host-only.  Number of regions of edge region_edge (a power of two,
 * >= 32) of a 3D grid: ceil(ny / edge) * ceil(nz / edge); at most 1024. */
int pcrit_region_count(int64_t nx, int64_t ny, int64_t nz, int region_edge,
                       int *n_host);

/* The progressive classification of pcrit_progressive (no list codes, no
 * re-classification count) with a timeline: the leading small levels run in
 * two launches (levels of at most 2^18 vertices, then the others up to
 * 2^22), and each later level that takes the quad tiles is classified region
 * by region in the chosen order, the wave that finishes a region's last
 * tile recording the GPU clock.  Times count from a first stamp that the GPU
 * takes after a 0.3 ms wait, by which time the host has queued the call's
 * kernels (so host launch latency stays out of them).  The call synchronises
 * at its end.
 *   order_mode        0: regions in id order; 1: rank_host[r] is the
 *                     position of region r (a permutation); 2: learned, from
 *                     the network with parameters mlp_params (device), run
 *                     on the GPU before the first region-refined level (the
 *                     scores of level pcrit_mlp_feature_level, ties by id);
 *                     then rank_host, if not NULL, receives the positions
 *                     used (the identity if no level is refined by regions)
 *   level_offsets_host  as for pcrit_progressive (k_max+2 entries)
 *   level_ms_host     k_max+1 doubles: milliseconds from the first stamp
 *                     until level k's list is complete (index i = k_max - k)
 *   region_ms_host    (k_max+1) x n_regions doubles: [i][r] = milliseconds
 *                     until level k of region r was classified (for levels
 *                     not refined by regions, the level's list time)
 * Errors as pcrit_progressive; PCRIT_E_ARG for 2D grids, a bad order or
 * edge. */
int pcrit_progressive_timeline(pcrit_ctx *ctx, void *hip_stream, const float *field,
                               int64_t nx, int64_t ny, int64_t nz, uint8_t *codes,
                               uint32_t *crit, int64_t crit_capacity, int region_edge,
                               int order_mode, int32_t *rank_host,
                               const float *mlp_params, int64_t *level_offsets_host,
                               double *level_ms_host, double *region_ms_host);

/* ------------------------------------------------------------------------
 * Batches of independent fields.
 *
 * Every field of the batch is classified at level 0 exactly as
 * pcrit_classify would (Section 3.1, ties by index within the field), but
 * groups of up to 16 fields share one classification launch and one
 * compaction launch, so many small fields do not pay a launch pair each.
 * ---------------------------------------------------------------------- */
#define PCRIT_MAX_BATCH_FIELDS (1 << 20)

typedef struct pcrit_batch_field {
  const float *field;  /* device, float32 C order [z][y][x], 4-byte aligned */
  int64_t nx, ny, nz;  /* as for pcrit_classify; nz == 1: 2D */
  uint8_t *codes;      /* device, nx*ny*nz bytes (written at every vertex) */
} pcrit_batch_field;

/* Classify n_fields fields (1 .. PCRIT_MAX_BATCH_FIELDS, all 3D or all 2D,
 * else PCRIT_E_ARG) described by fields_host (host array).
 *   crit, crit_codes, crit_capacity  one list for the whole batch: field i's
 *                     ascending critical indices (field-local, uint32) are
 *                     crit[off[i] .. off[i+1]); entries past the capacity
 *                     are not written; crit_codes may be NULL
 *   offsets_dev       device, n_fields+1 int64, or NULL: the list offsets,
 *                     written on the stream (off[0] = 0)
 *   offsets_host      host, n_fields+1 int64, or NULL: non-NULL makes the
 *                     call wait for the stream and copy the offsets
 * Errors: as pcrit_classify for each field's sizes (the first failing
 * field's status); with offsets_host, PCRIT_E_NAN if any field has a NaN
 * sample and PCRIT_E_CAPACITY if off[n_fields] > crit_capacity (the
 * offsets then hold the required sizes).  Without offsets_host the call
 * launches kernels only (no allocation once the context's scratch has grown
 * to the batch, no memset, no wait), so it can be captured in a HIP graph;
 * calls that overlap on one context race (they share its scratch).  With
 * more than 16 fields a group's compaction runs on the context's second
 * stream while the next group is classified on hip_stream (events fork and
 * join the streams; the call's work still ends on hip_stream). */
int pcrit_classify_batch(pcrit_ctx *ctx, void *hip_stream, int n_fields,
                         const pcrit_batch_field *fields_host, uint32_t *crit,
                         uint8_t *crit_codes, int64_t crit_capacity,
                         int64_t *offsets_host, int64_t *offsets_dev);

/* Batch launch configuration (per context): `group` fields share one
 * classification launch and one compaction launch (1 ..
 * PCRIT_BATCH_GROUP_MAX; 0 = the default, 16), and each field's tiles are
 * as deep as still gives `want_tiles` wave tiles per field (64 .. 2^20;
 * 0 = the default, 512).  Results do not depend on it; only the time
 * does.  PCRIT_E_ARG for values out of range. */
#define PCRIT_BATCH_GROUP_MAX 16
int pcrit_set_batch_config(pcrit_ctx *ctx, int group, int64_t want_tiles);
int pcrit_get_batch_config(pcrit_ctx *ctx, int *group, int64_t *want_tiles);

/* Autotuner of the batch configuration: times pcrit_classify_batch on the
 * caller's fields and buffers (arguments as there) for each of
 * PCRIT_BATCH_TUNE_CANDIDATES configurations, group in {8, 16} (outer)
 * times want_tiles in {128, 256, 512, 1024, 2048, 4096} (inner), each after one
 * untimed call, over `reps` calls (1 .. 100) between two HIP events on the
 * stream, and keeps the fastest in the context for later batch calls.
 * times_ms_host (NULL or PCRIT_BATCH_TUNE_CANDIDATES doubles) receives the
 * time per call of each candidate in that order; group_out and want_out
 * (NULL or one each) the choice.  A first call with the context's
 * configuration checks the batch (its errors are returned, the
 * configuration is then unchanged); a last call with the chosen one leaves
 * the batch's lists and codes in the caller's buffers.  The call
 * waits for the stream; not for graph capture (scratch may grow). */
#define PCRIT_BATCH_TUNE_CANDIDATES 12
int pcrit_batch_autotune(pcrit_ctx *ctx, void *hip_stream, int n_fields,
                         const pcrit_batch_field *fields_host, uint32_t *crit,
                         uint8_t *crit_codes, int64_t crit_capacity, int reps,
                         double *times_ms_host, int *group_out, int64_t *want_out);

/* ------------------------------------------------------------------------
 * Order field and extremum lists (the
 * inputs of the paper's simplification).
 * ---------------------------------------------------------------------- */

/* The order field of Section 4.1: every vertex ranked by (value, memory
 * index), ties by index, -0 == +0:
 *   rank[i] = #{ j : f[j] < f[i] or (f[j] == f[i] and j < i) },
 *   sorted[r] = the vertex of rank r
 * (device, N uint32 each, caller-owned).  A radix sort on the GPU; the call
 * waits for the stream.  PCRIT_E_NAN if a sample is NaN (outputs then
 * unspecified).  Dims as for pcrit_classify (N <= 2^32 - 1). */
int pcrit_order_field(pcrit_ctx *ctx, void *hip_stream, const float *field, int64_t nx,
                      int64_t ny, int64_t nz, uint32_t *rank, uint32_t *sorted);

/* The extremum lists of full-resolution codes (as written by
 * pcrit_classify at level 0): minima (empty lower link, code & 7 == 0), then
 * maxima (empty upper link, code & 0x38 == 0), each ascending, into out
 * (device, capacity entries; entries past it are not written).
 * counts_host[0] = minima, counts_host[1] = maxima; PCRIT_E_CAPACITY if
 * their sum exceeds the capacity.  The call waits for the stream. */
int pcrit_extrema(pcrit_ctx *ctx, void *hip_stream, const uint8_t *codes, int64_t nx,
                  int64_t ny, int64_t nz, uint32_t *out, int64_t capacity, int64_t *counts_host);

/* ------------------------------------------------------------------------
 * Step 1 of localized topological simplification: the superlevel /
 * sublevel set propagation from each extremum (Section 4.2, step 1) with
 * the persistence test of Section 4.5, on its own or merged at saddles
 * (Section 4.4).
 * ---------------------------------------------------------------------- */
#define PCRIT_LTS_SADDLE 0     /* stopped at the saddle where it meets another component */
#define PCRIT_LTS_PERSISTENT 1 /* value difference to the extremum exceeded epsilon */
#define PCRIT_LTS_BUDGET 2     /* component or waiting set outgrew the budget */
#define PCRIT_LTS_INVALID 3    /* the listed index is not a vertex of the grid */
#define PCRIT_LTS_MAX_VISITED 32
#define PCRIT_LTS_MAX_FRONTIER 128

/* For each extremum ext[i] (device, n_extrema uint32 full-resolution
 * indices; maxima when maxima != 0, else minima) of the field (device,
 * float32, nx*ny*nz) with order field rank (device, as pcrit_order_field
 * writes it): grow the extremum's component one vertex at a time, always
 * taking the largest vertex in the order (the smallest for minima) adjacent
 * to it, among the Freudenthal neighbours of pcrit_classify.  Stop when the
 * vertex just taken
 *   - differs from the extremum by more than epsilon in value (float32,
 *     f(m) - f(v) for maxima, f(v) - f(m) for minima): PCRIT_LTS_PERSISTENT;
 *   - has a larger (smaller) neighbour outside the component: it is the
 *     saddle, PCRIT_LTS_SADDLE;
 * or PCRIT_LTS_BUDGET once the component holds max_visited vertices (2 ..
 * PCRIT_LTS_MAX_VISITED) or more than max_frontier (14 ..
 * PCRIT_LTS_MAX_FRONTIER) vertices wait outside it.  Outputs (device,
 * n_extrema entries each): status (uint8), saddle (int32 index, -1 unless
 * a saddle stop) and visited (uint16, vertices taken, the extremum
 * included).  Every extremum propagates on its own (propagations that meet
 * at a saddle are not merged; pcrit_lts_merged merges them).
 * Asynchronous: kernels only, no wait.
 * PCRIT_E_ARG for NULL or misaligned pointers, a NaN epsilon or budgets
 * out of range; dims as for pcrit_classify. */
int pcrit_lts_propagate(pcrit_ctx *ctx, void *hip_stream, const float *field,
                        const uint32_t *rank, int64_t nx, int64_t ny, int64_t nz,
                        const uint32_t *extrema, int64_t n_extrema, int maxima, float epsilon,
                        int max_visited, int max_frontier, uint8_t *status, int32_t *saddle,
                        uint16_t *visited);

/* Merged propagations (Sections 4.4 and 4.5): the propagations of the
 * listed extrema (distinct vertices; maxima when maxima != 0, else minima)
 * grow as in pcrit_lts_propagate, each led by its extremum, but meet at
 * saddles.  A propagation that stops at a saddle s adds the higher (lower,
 * for minima) neighbours of s it holds to s's arrival count; the one whose
 * addition makes the count equal s's number of such neighbours goes on
 * from s with the union of every component that arrived there, led by the
 * largest (smallest) of their leaders, whose value the persistence test
 * then uses.  The leaders of the other arrived components are paired with
 * s: status PCRIT_LTS_SADDLE, saddle s, visited = the size of the component
 * they led.  A leader whose component stopped at a saddle that no later
 * arrival completes stays paired with it.  PCRIT_LTS_PERSISTENT when the
 * persistence test stops the propagation it leads (or when it takes the
 * whole grid); PCRIT_LTS_BUDGET when that propagation outgrows the budgets
 * of pcrit_lts_propagate, a merge included (union of max_visited vertices
 * or more, or more than max_frontier waiting; visited is then the union's
 * size); PCRIT_LTS_INVALID for an index outside the grid or a vertex with a
 * neighbour later in the order (earlier, for minima).  With every extremum
 * listed and budgets that no propagation reaches, the extrema paired with
 * a saddle are those whose persistence (elder rule, in value) is at most
 * epsilon.  The result does not depend on which propagation arrives last;
 * with a listed vertex repeated it is unspecified.  The context keeps
 * scratch of about 690 bytes per listed extremum (grown on demand, with a
 * device synchronisation).  Asynchronous otherwise: kernels only (a start
 * kernel and max_visited merge rounds), no wait.
 * Errors as for pcrit_lts_propagate; PCRIT_E_ARG also for more than 2^30
 * extrema, PCRIT_E_OOM if the scratch cannot be allocated. */
int pcrit_lts_merged(pcrit_ctx *ctx, void *hip_stream, const float *field, const uint32_t *rank,
                     int64_t nx, int64_t ny, int64_t nz, const uint32_t *extrema,
                     int64_t n_extrema, int maxima, float epsilon, int max_visited,
                     int max_frontier, uint8_t *status, int32_t *saddle, uint16_t *visited);

#ifdef __cplusplus
}
#endif

#endif /* PCRIT_H */
