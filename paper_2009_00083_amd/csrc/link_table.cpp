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

void build_quad_table3(const uint8_t *table3, uint8_t *quad) {
  // where each neighbour offset of the link-pattern table sits in the quad
  // index: positive direction j (its bit is 1 iff the neighbour is lower)
  // or negative direction j (bit 8 + j, 1 iff the neighbour is upper)
  int dir[14], neg[14];
  for (int k = 0; k < 14; k++) {
    dir[k] = -1;
    for (int j = 0; j < 7; j++) {
      if (kQD[j][0] == kOff3[k][0] && kQD[j][1] == kOff3[k][1] && kQD[j][2] == kOff3[k][2]) {
        dir[k] = j;
        neg[k] = 0;
      }
      if (kQD[j][0] == -kOff3[k][0] && kQD[j][1] == -kOff3[k][1] && kQD[j][2] == -kOff3[k][2]) {
        dir[k] = j;
        neg[k] = 1;
      }
    }
  }
  for (unsigned i = 0; i < (unsigned)kQuadTableSize; i++) {
    const unsigned p = i & 0x7Fu, n = (i >> 8) & 0x7Fu;
    unsigned m = 0;  // bit k = 1 iff neighbour k comes after the vertex
    for (int k = 0; k < 14; k++) {
      const unsigned upper = neg[k] ? (n >> dir[k]) & 1u : ((p >> dir[k]) & 1u) ^ 1u;
      m |= upper << k;
    }
    quad[i] = (i & 0x8000u) ? 0 : table3[m];
  }
  // x-boundary codes: the absent neighbours forced upper, then lower (the
  // rule the kernels apply to other boundary vertices), by index without
  // the absent bits
  auto boundary = [&](unsigned idx, unsigned A) {
    const unsigned base = idx & ~A;
    const unsigned eL = quad[base | (A & kQNeg)], eU = quad[base | (A & kQPos)];
    const unsigned holes = ((eL >> 3) > 1u) | ((eU & 7u) > 1u);
    return (uint8_t)((eL & 7u) | (eU & 0x38u) | 0x40u | (holes << 7));
  };
  uint8_t *txl = quad + kQuadTableSize, *txh = quad + kQuadTableSize + 1024;
  for (unsigned c = 0; c < 1024; c++) {
    txl[c] = boundary((c & 0x7Fu) | ((c >> 7) << 12), quad_side(0, -1));
    txh[c] = boundary(((c & 7u) << 4) | ((c >> 3) << 8), quad_side(0, 1));
  }
}

}  // namespace pcrit
