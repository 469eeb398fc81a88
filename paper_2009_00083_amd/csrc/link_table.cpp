// Link-pattern tables for the classification kernels (host side).
//
// The link of an interior grid vertex v (Section 3.1: faces of the star
// simplices that do not contain v) has the neighbours of v as vertices.  In
// the grid triangulation used here (cubes cut into the six tetrahedra along
// the (1,1,1) diagonal, squares along (1,1)) a set of grid points spans a
// simplex exactly when all pairwise differences are neighbour offsets, so
// two neighbours u, w of v are joined by a link edge iff w - u is itself a
// neighbour offset.  The components of the lower (upper) link are therefore
// the components of that graph restricted to the neighbours below (above) v.
// The table stores, for every polarity mask, the component counts of the
// 0-bits and of the 1-bits.
#include "pcrit_internal.h"

namespace pcrit {
namespace {

template <int D>
bool is_offset(const int *d) {
  bool any = false, nonneg = true, nonpos = true;
  for (int a = 0; a < D; a++) {
    if (d[a] < -1 || d[a] > 1) return false;
    any |= d[a] != 0;
    nonneg &= d[a] >= 0;
    nonpos &= d[a] <= 0;
  }
  return any && (nonneg || nonpos);
}

// Number of connected components of vertex set `set` in the graph `adj`.
int count_components(unsigned set, const unsigned *adj) {
  int count = 0;
  while (set) {
    unsigned comp = set & (~set + 1u);  // lowest vertex as seed
    unsigned prev = 0;
    while (comp != prev) {
      prev = comp;
      for (unsigned r = comp; r; r &= r - 1) {
        int i = __builtin_ctz(r);
        comp |= adj[i] & set;
      }
    }
    set &= ~comp;
    count++;
  }
  return count;
}

template <int D, int N>
void build(const int (*off)[D], uint8_t *table) {
  unsigned adj[N];
  for (int i = 0; i < N; i++) {
    adj[i] = 0;
    for (int j = 0; j < N; j++) {
      int d[D];
      for (int a = 0; a < D; a++) d[a] = off[j][a] - off[i][a];
      if (is_offset<D>(d)) adj[i] |= 1u << j;
    }
  }
  const unsigned all = (1u << N) - 1u;
  for (unsigned m = 0; m <= all; m++) {
    int c0 = count_components(all & ~m, adj);
    int c1 = count_components(m, adj);
    table[m] = (uint8_t)(c0 | (c1 << 3));
  }
}

}  // namespace

void build_link_table3(uint8_t *table) { build<3, 14>(kOff3, table); }
void build_link_table2(uint8_t *table) { build<2, 6>(kOff2, table); }

}  // namespace pcrit
