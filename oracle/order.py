"""CPU oracle of the order field and the extremum lists (test
infrastructure: only the tests and bench.py's CPU baseline use it; the GPU
library never imports it).

The order field of Section 4.1 ranks every vertex by its value, ties by
memory index; -0 and +0 are equal values (IEEE comparison).  Written with
numpy: a stable sort of the values (numpy's stable sort keeps equal values
in index order), then rank[sorted[r]] = r.  The extremum lists are the
vertices whose lower (upper) link is empty, read from the classification
codes (bits 0-2: lower-link components, bits 3-5: upper-link components).

Pins (``tests/test_oracle_order.py``): brute-force ranks by pairwise
comparison on small inputs; closed forms of linear and constant fields and
of signed zeros; the classification of a field equals that of its order
field; extremum lists of linear fields and of hand-made code arrays.
"""
from __future__ import annotations

import numpy as np


def order_field(f):
    """(rank, sorted): rank[i] = position of vertex i in the order of
    (value, index); sorted[r] = vertex of rank r.  Raises on NaN."""
    v = np.asarray(f, dtype=np.float32).ravel()
    if np.isnan(v).any():
        raise ValueError("NaN sample")
    v = v.astype(np.float64) + 0.0  # -0 + 0 = +0: equal values compare equal anyway
    srt = np.argsort(v, kind="stable")
    rank = np.empty(v.size, np.int64)
    rank[srt] = np.arange(v.size)
    return rank.astype(np.uint32), srt.astype(np.uint32)


def extrema(codes):
    """(minima, maxima): ascending full-resolution indices of the vertices
    with no lower (upper) link component."""
    c = np.asarray(codes, dtype=np.uint8).ravel()
    return (np.flatnonzero((c & 0x07) == 0).astype(np.uint32),
            np.flatnonzero((c & 0x38) == 0).astype(np.uint32))
