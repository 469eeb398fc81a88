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
 *     plane must hold at most 2^30 samples (nx*ny in 3D, nx in 2D), since
 *     the kernels address it with 32-bit byte offsets;
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
                                 plane of more than 2^30 samples */
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
 * level's list complete before the next level starts.  A vertex already
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
 *   level_ms_host host, k_max+1 entries or NULL: milliseconds from the first
 *                 enqueued kernel to the completion of level k, at index
 *                 i = k_max - k (stream-event timing; NULL records no
 *                 events).  Levels whose work shares one launch (see below)
 *                 report the same time
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

#ifdef __cplusplus
}
#endif

#endif /* PCRIT_H */
