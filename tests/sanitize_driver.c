/* Host-code driver for the sanitizer build (tests/test_sanitize.py): runs the
 * oracle (oracle/pcrit_oracle.c) and the library's host-only preview metric
 * (csrc/metrics.cpp) over small grids of every kind -- random, tie-heavy,
 * constant, with infinities and NaN, 2D and 3D, every level, restricted
 * ranges, small capacities, one and several threads -- and over bad
 * arguments, so that AddressSanitizer and UndefinedBehaviorSanitizer see
 * every path.  Exits non-zero on an inconsistent result. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_classify(const float *f, int64_t nx, int64_t ny, int64_t nz, int level,
                    int64_t slow_begin, int64_t slow_end, uint8_t *codes, int8_t *chi_lower,
                    int8_t *chi_upper, uint32_t *crit, int64_t crit_cap, int64_t *crit_count,
                    int nthreads);
int oracle_level_dims(int64_t nx, int64_t ny, int64_t nz, int level, int64_t *m_out);
int oracle_vertex_detail(const float *f, int64_t nx, int64_t ny, int64_t nz, int level,
                         int64_t count, const int64_t *coords, int *out);
int oracle_classify_link(int nv, const int *lower, int ne, const int *edges, int nt,
                         const int *tris, int link_dim, int link_closed, int *out);
int pcrit_preview_f1(int64_t nx, int64_t ny, int64_t nz, int level, const uint32_t *preview,
                     const uint8_t *preview_codes, int64_t n_preview, const uint32_t *exact,
                     const uint8_t *exact_codes, int64_t n_exact, double *f1,
                     int64_t *matches);
int pcrit_preview_f1_levels(int64_t nx, int64_t ny, int64_t nz, const uint32_t *preview,
                            const uint8_t *preview_codes, const uint8_t *preview_levels,
                            int64_t n_preview, const uint32_t *exact,
                            const uint8_t *exact_codes, int64_t n_exact, double *f1,
                            int64_t *matches);

static uint64_t rng_state = 88172645463325252ull;
static uint32_t rnd(void) {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (uint32_t)(rng_state >> 16);
}

static int failures = 0;
#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      failures++;                                                   \
    }                                                               \
  } while (0)

static void fill(float *f, int64_t n, int kind) {
  for (int64_t i = 0; i < n; i++) {
    switch (kind) {
      case 0: f[i] = (float)(rnd() % 100000) / 1000.0f; break;   /* random */
      case 1: f[i] = (float)(rnd() % 3); break;                   /* ties */
      case 2: f[i] = 0.5f; break;                                 /* constant */
      case 3: {                                                   /* specials */
        static const float v[6] = {0.0f, -0.0f, INFINITY, -INFINITY, 1.0f, -1.0f};
        f[i] = v[rnd() % 6];
        break;
      }
      default: f[i] = (float)i; break;                            /* linear */
    }
  }
}

static void run_grid(int64_t nx, int64_t ny, int64_t nz) {
  const int64_t n = nx * ny * nz;
  float *f = malloc(sizeof(float) * (size_t)n);
  uint8_t *codes = malloc((size_t)n);
  uint32_t *crit = malloc(sizeof(uint32_t) * (size_t)n);
  int8_t *chl = malloc((size_t)n), *chu = malloc((size_t)n);
  for (int kind = 0; kind < 5; kind++) {
    fill(f, n, kind);
    for (int level = 0; level < 8; level++) {
      int64_t m[3];
      if (oracle_level_dims(nx, ny, nz, level, m)) break;
      const int64_t nl = m[0] * m[1] * m[2];
      for (int threads = 1; threads <= 3; threads += 2) {
        int64_t cnt = -1;
        memset(codes, 0, (size_t)n);
        int st = oracle_classify(f, nx, ny, nz, level, 0, -1, codes, chl, chu, crit, nl, &cnt,
                                 threads);
        CHECK(st == 0);
        CHECK(cnt >= 0 && cnt <= nl);
        int64_t ncrit = 0;
        for (int64_t i = 0; i < cnt; i++) {
          CHECK(crit[i] < (uint64_t)n);
          if (i) CHECK(crit[i] > crit[i - 1]);
        }
        /* the list is exactly the critical codes of the level */
        const int64_t s = (int64_t)1 << level;
        for (int64_t z = 0; z < nz; z += (nz > 1 ? s : 1))
          for (int64_t y = 0; y < ny; y += s)
            for (int64_t x = 0; x < nx; x += s) ncrit += (codes[(z * ny + y) * nx + x] & 0xBF) != 9;
        CHECK(ncrit == cnt);
        /* a restricted range and a capacity too small */
        const int slow = nz > 1 ? 2 : 1;
        int64_t c2 = -1;
        st = oracle_classify(f, nx, ny, nz, level, 1, m[slow] - 1, codes, NULL, NULL, crit, 1,
                             &c2, threads);
        CHECK(st == 0 || st == -4);
        CHECK(c2 >= 0 && c2 <= cnt);
      }
      /* per-vertex detail of a few vertices */
      int64_t coords[3 * 4];
      for (int k = 0; k < 4; k++) {
        coords[3 * k] = rnd() % m[0];
        coords[3 * k + 1] = rnd() % m[1];
        coords[3 * k + 2] = rnd() % m[2];
      }
      int out[12 * 4];
      CHECK(oracle_vertex_detail(f, nx, ny, nz, level, 4, coords, out) == 0);
    }
  }
  /* NaN on the level */
  fill(f, n, 0);
  f[n / 2] = NAN;
  int64_t cnt = 0;
  CHECK(oracle_classify(f, nx, ny, nz, 0, 0, -1, codes, NULL, NULL, crit, n, &cnt, 2) == -5);
  /* bad arguments */
  CHECK(oracle_classify(NULL, nx, ny, nz, 0, 0, -1, codes, NULL, NULL, crit, n, &cnt, 1) < 0);
  CHECK(oracle_classify(f, nx, ny, nz, 30, 0, -1, codes, NULL, NULL, crit, n, &cnt, 1) < 0);
  free(f);
  free(codes);
  free(crit);
  free(chl);
  free(chu);
}

static void run_metric(int64_t nx, int64_t ny, int64_t nz) {
  const int64_t n = nx * ny * nz;
  for (int rep = 0; rep < 20; rep++) {
    const int64_t np = rnd() % 40, ne = rnd() % 40;
    uint32_t *p = malloc(sizeof(uint32_t) * (size_t)(np + 1));
    uint32_t *e = malloc(sizeof(uint32_t) * (size_t)(ne + 1));
    uint8_t *pc = malloc((size_t)(np + 1)), *ec = malloc((size_t)(ne + 1));
    uint8_t *pl = malloc((size_t)(np + 1));
    static const uint8_t kinds[4] = {0x09, 0x00, 0x12, 0x38};
    for (int64_t i = 0; i < np; i++) {
      p[i] = rnd() % (uint32_t)n;
      pc[i] = kinds[rnd() % 4];
      pl[i] = (uint8_t)(rnd() % 3);
    }
    for (int64_t i = 0; i < ne; i++) {
      e[i] = rnd() % (uint32_t)n;
      ec[i] = kinds[1 + rnd() % 3];
    }
    double f1 = -1;
    int64_t mt = -1;
    CHECK(pcrit_preview_f1(nx, ny, nz, (int)(rnd() % 3), p, pc, np, e, ec, ne, &f1, &mt) == 0);
    CHECK(f1 >= 0.0 && f1 <= 1.0 && mt >= 0 && mt <= np && mt <= ne);
    CHECK(pcrit_preview_f1_levels(nx, ny, nz, p, pc, pl, np, e, ec, ne, &f1, &mt) == 0);
    CHECK(f1 >= 0.0 && f1 <= 1.0);
    /* an index past the grid is an argument error */
    if (np) {
      p[0] = (uint32_t)n;
      CHECK(pcrit_preview_f1(nx, ny, nz, 0, p, pc, np, e, ec, ne, &f1, &mt) < 0);
    }
    free(p);
    free(e);
    free(pc);
    free(ec);
    free(pl);
  }
}

int main(void) {
  static const int64_t shapes[][3] = {{5, 6, 7}, {9, 4, 3}, {2, 2, 2}, {17, 3, 2},
                                      {7, 9, 1}, {2, 2, 1}, {33, 5, 1}};
  for (size_t k = 0; k < sizeof(shapes) / sizeof(shapes[0]); k++) {
    run_grid(shapes[k][0], shapes[k][1], shapes[k][2]);
    run_metric(shapes[k][0], shapes[k][1], shapes[k][2]);
  }
  /* a hand-written link: a 4-cycle with two opposite lower vertices */
  const int lower[4] = {1, 0, 1, 0}, edges[8] = {0, 1, 1, 2, 2, 3, 3, 0};
  int out[6];
  CHECK(oracle_classify_link(4, lower, 4, edges, 0, NULL, 1, 1, out) == 1);
  CHECK(oracle_classify_link(-1, lower, 4, edges, 0, NULL, 1, 1, out) < 0);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("sanitized host code: all checks passed\n");
  return 0;
}
