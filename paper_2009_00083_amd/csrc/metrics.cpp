// Preview quality metric (host): F1 of a coarse level's critical list
// against the exact list, with one-to-one greedy matching by distance.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/pcrit.h"

namespace {

// 1 minimum, 2 maximum, 3 saddle (any other critical code), 0 regular
inline unsigned char point_type(unsigned char code) {
  const int nl = code & 7, nu = (code >> 3) & 7;
  if (nl == 0) return 1;
  if (nu == 0) return 2;
  if (nl == 1 && nu == 1 && !(code & 0x80)) return 0;
  return 3;
}

// Preview points carry their own level (tolerance 2^level); `levels` may be
// null, then every point has level `level`.
int preview_f1(int64_t nx, int64_t ny, int64_t nz, int level, const uint8_t *levels,
               const uint32_t *preview, const uint8_t *preview_codes, int64_t n_preview,
               const uint32_t *exact, const uint8_t *exact_codes, int64_t n_exact,
               double *f1, int64_t *matches_out) {
  if (!f1 || n_preview < 0 || n_exact < 0 || level < 0 || level > 30 ||
      (n_preview && (!preview || !preview_codes)) ||
      (n_exact && (!exact || !exact_codes)))
    return PCRIT_E_ARG;
  if (levels) {
    level = 0;
    for (int64_t i = 0; i < n_preview; i++) {
      if (levels[i] > 30) return PCRIT_E_ARG;
      level = std::max(level, (int)levels[i]);
    }
  }
  if (nx < 2 || ny < 2 || nz < 1) return PCRIT_E_DIMS;
  const int64_t n = nx * ny * nz;
  if (n > 4294967295ll) return PCRIT_E_DIMS;
  if (n_preview + n_exact == 0) {
    *f1 = 1.0;
    if (matches_out) *matches_out = 0;
    return PCRIT_OK;
  }
  std::vector<unsigned char> etype((size_t)n, 0);
  for (int64_t i = 0; i < n_exact; i++) {
    if (exact[i] >= (uint64_t)n) return PCRIT_E_ARG;
    etype[exact[i]] = point_type(exact_codes[i]);
  }
  std::vector<unsigned char> pmatched((size_t)n_preview, 0);
  for (int64_t i = 0; i < n_preview; i++)
    if (preview[i] >= (uint64_t)n) return PCRIT_E_ARG;
  const int64_t D = (int64_t)1 << level;
  const int64_t dzmax = nz > 1 ? D : 0;
  int64_t matches = 0;
  // Greedy over pairs sorted by (distance, preview index, exact index):
  // distance classes in increasing order; inside a class the preview points
  // in increasing index, each taking its smallest-index free partner.
  for (int64_t d = 0; d <= D; d++) {
    for (int64_t i = 0; i < n_preview; i++) {
      if (pmatched[i]) continue;
      const int64_t p = preview[i];
      const unsigned char t = point_type(preview_codes[i]);
      if (!t) continue;
      if (levels && d > ((int64_t)1 << levels[i])) continue;
      const int64_t px = p % nx, py = (p / nx) % ny, pz = p / (nx * ny);
      bool found = false;
      const int64_t dz0 = -std::min(d, dzmax), dz1 = std::min(d, dzmax);
      for (int64_t dz = dz0; dz <= dz1 && !found; dz++) {
        const int64_t z = pz + dz;
        if (z < 0 || z >= nz) continue;
        const bool zfull = (dz == d || dz == -d);
        for (int64_t dy = -d; dy <= d && !found; dy++) {
          const int64_t y = py + dy;
          if (y < 0 || y >= ny) continue;
          const bool full = zfull || dy == d || dy == -d;
          const int64_t row = (z * ny + y) * nx;
          if (full) {
            for (int64_t dx = -d; dx <= d; dx++) {
              const int64_t x = px + dx;
              if (x < 0 || x >= nx) continue;
              if (etype[row + x] == t) {
                etype[row + x] = 0;  // taken
                found = true;
                break;
              }
            }
          } else {
            const int64_t xs[2] = {px - d, px + d};
            for (int j = 0; j < (d ? 2 : 1); j++) {
              const int64_t x = xs[j];
              if (x < 0 || x >= nx) continue;
              if (etype[row + x] == t) {
                etype[row + x] = 0;
                found = true;
                break;
              }
            }
          }
        }
      }
      if (found) {
        pmatched[i] = 1;
        matches++;
      }
    }
  }
  *f1 = 2.0 * (double)matches / (double)(n_preview + n_exact);
  if (matches_out) *matches_out = matches;
  return PCRIT_OK;
}

}  // namespace

extern "C" int pcrit_preview_f1(int64_t nx, int64_t ny, int64_t nz, int level,
                                const uint32_t *preview,
                                const uint8_t *preview_codes, int64_t n_preview,
                                const uint32_t *exact,
                                const uint8_t *exact_codes, int64_t n_exact,
                                double *f1, int64_t *matches_out) {
  return preview_f1(nx, ny, nz, level, nullptr, preview, preview_codes, n_preview, exact,
                    exact_codes, n_exact, f1, matches_out);
}

extern "C" int pcrit_preview_f1_levels(int64_t nx, int64_t ny, int64_t nz,
                                       const uint32_t *preview,
                                       const uint8_t *preview_codes,
                                       const uint8_t *preview_levels_host, int64_t n_preview,
                                       const uint32_t *exact, const uint8_t *exact_codes,
                                       int64_t n_exact, double *f1, int64_t *matches_out) {
  if (n_preview && !preview_levels_host) return PCRIT_E_ARG;
  return preview_f1(nx, ny, nz, 0, preview_levels_host ? preview_levels_host : (const uint8_t *)"",
                    preview, preview_codes, n_preview, exact, exact_codes, n_exact, f1,
                    matches_out);
}
