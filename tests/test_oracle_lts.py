"""Pins of the LTS Step 1 oracle (superlevel / sublevel set propagation
from each extremum, Sections 4.2 and 4.5): an independent breadth-first
definition of the component, the saddle's properties, the persistence rule,
closed forms, and the symmetry of minima and maxima."""
import numpy as np
import pytest

import fieldgen
import oracle
from oracle import lts
from oracle.order import extrema, order_field


def _fields():
    yield fieldgen.iid_field((9, 8, 7), 3)
    yield fieldgen.gaussian_field((12, 10, 9), 4, 5, noise=("uniform", 2e-2))
    yield fieldgen.iid_field((13, 11), 5)
    yield fieldgen.tie_field((8, 9, 6), 6, 3)


@pytest.mark.parametrize("maxima", [True, False])
def test_saddle_stop_is_the_superlevel_component(maxima):
    """For every stop at a saddle s: the vertices taken are exactly the
    component of the strict superlevel set {u : key(u) > key(s)} that
    contains the extremum, together with s (at the level of s itself the
    component joins the one beyond s); s is the smallest of them and has a
    larger neighbour outside."""
    checked = 0
    for f in _fields():
        codes = oracle.classify(f).codes
        mn, mx = extrema(codes)
        rank, _ = order_field(f)
        key = rank.astype(np.int64) if maxima else rank.size - 1 - rank.astype(np.int64)
        for m in (mx if maxima else mn):
            st, s, comp = lts.propagate_set(f, key, f.shape, int(m), np.inf, 400, 4000, maxima)
            assert st in (lts.SADDLE, lts.BUDGET)
            if st != lts.SADDLE:
                continue
            assert comp == lts.superlevel_component(f.shape, key, int(m), key[s] + 1) | {s}
            assert key[s] == min(key[c] for c in comp)
            assert any(u not in comp and key[u] > key[s] for u in lts.neighbours(f.shape, s))
            checked += 1
    assert checked > 50


def test_persistence_rule():
    """With a finite epsilon an extremum stops at the same saddle if the
    value difference to it is at most epsilon, and is persistent
    otherwise (the difference grows along the propagation)."""
    f = fieldgen.gaussian_field((12, 11, 10), 8, 6, noise=("uniform", 3e-2))
    codes = oracle.classify(f).codes
    _, mx = extrema(codes)
    st0, sd0, _ = lts.propagate_all(f, mx, np.inf, max_visited=500, max_frontier=5000)
    fv = f.ravel()
    for eps in (0.0, 0.01, 0.03, 0.1):
        st, sd, _ = lts.propagate_all(f, mx, eps, max_visited=500, max_frontier=5000)
        for i, m in enumerate(mx):
            if st0[i] != lts.SADDLE:
                continue
            d = np.float32(fv[m] - fv[sd0[i]])
            if d <= np.float32(eps):
                assert st[i] == lts.SADDLE and sd[i] == sd0[i]
            else:
                assert st[i] == lts.PERSISTENT and sd[i] == -1


def test_two_bumps_closed_form():
    """2D, two peaks on the line y = 3 joined through a pass at x = 5: the
    lower peak's propagation stops at the pass, after taking the 21
    vertices of columns 2..4 and the pass itself."""
    g = np.array([0, 0.5, 1, 0.7, 0.6, 0.5, 1.2, 1.6, 2, 1.5, 1], np.float32)
    ny, cy = 7, 3
    y = np.arange(ny)[:, None]
    f = (g[None, :] - 0.01 * np.abs(y - cy)).astype(np.float32)
    rank, _ = order_field(f)
    st, s, comp = lts.propagate_set(f, rank.astype(np.int64), f.shape, cy * 11 + 2, np.inf, 100, 1000)
    assert st == lts.SADDLE and s == cy * 11 + 5 and len(comp) == 22
    # the higher peak meets no larger component: it runs to the budget
    st2, s2, comp2 = lts.propagate_set(f, rank.astype(np.int64), f.shape, cy * 11 + 8, np.inf, 30, 1000)
    assert st2 == lts.BUDGET and s2 == -1 and len(comp2) == 30
    # with epsilon below the height above the pass (0.5) the lower peak is
    # persistent, at or above it not
    assert lts.propagate(f, rank.astype(np.int64), f.shape, cy * 11 + 2, 0.49, 100, 1000)[0] == lts.PERSISTENT
    assert lts.propagate(f, rank.astype(np.int64), f.shape, cy * 11 + 2, 0.5, 100, 1000)[:2] == (lts.SADDLE, cy * 11 + 5)


def test_single_bump_has_no_saddle():
    z, y, x = np.meshgrid(np.arange(7), np.arange(8), np.arange(9), indexing="ij")
    f = -((x - 4.2) ** 2 + (y - 3.7) ** 2 + (z - 3.1) ** 2).astype(np.float32)
    codes = oracle.classify(f).codes
    _, mx = extrema(codes)
    assert len(mx) == 1
    st, sd, vi = lts.propagate_all(f, mx, np.inf, max_visited=40, max_frontier=1000)
    assert st[0] == lts.BUDGET and sd[0] == -1 and vi[0] == 40


def test_minima_are_maxima_of_negated_field():
    f = fieldgen.iid_field((10, 9, 8), 11)  # no equal values: the orders reverse exactly
    mn, _ = extrema(oracle.classify(f).codes)
    _, mx_neg = extrema(oracle.classify(-f).codes)
    assert np.array_equal(mn, mx_neg)
    a = lts.propagate_all(f, mn, 0.05, maxima=False)
    b = lts.propagate_all(-f, mx_neg, 0.05, maxima=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_budget_limits():
    f = fieldgen.gaussian_field((14, 12, 10), 2, 3, noise=("uniform", 1e-4))
    _, mx = extrema(oracle.classify(f).codes)
    st, sd, vi = lts.propagate_all(f, mx, np.inf, max_visited=8, max_frontier=64)
    assert np.all(vi <= 8)
    assert np.all((st == lts.BUDGET) | (st == lts.SADDLE))
    assert np.all(sd[st == lts.BUDGET] == -1)


def test_neighbourhood_matches_the_classifier():
    """The propagation's neighbours are the link vertices of the classifier
    (its C code has its own offsets): a vertex whose neighbours are all
    smaller (larger) in the order is exactly a maximum (minimum) of the
    codes, in 3D and 2D, boundary vertices included."""
    for f in (fieldgen.iid_field((7, 6, 5), 21), fieldgen.iid_field((9, 8), 22),
              fieldgen.tie_field((6, 7, 5), 23, 2)):
        mn, mx = extrema(oracle.classify(f).codes)
        rank, _ = order_field(f)
        top = [v for v in range(f.size)
               if all(rank[u] < rank[v] for u in lts.neighbours(f.shape, v))]
        bottom = [v for v in range(f.size)
                  if all(rank[u] > rank[v] for u in lts.neighbours(f.shape, v))]
        assert np.array_equal(np.array(top, np.uint32), mx)
        assert np.array_equal(np.array(bottom, np.uint32), mn)
        # and the neighbourhood is symmetric, 14 (6) vertices inside
        for v in range(f.size):
            for u in lts.neighbours(f.shape, v):
                assert v in lts.neighbours(f.shape, u)
        centre = int(np.ravel_multi_index(tuple(n // 2 for n in f.shape), f.shape))
        assert len(lts.neighbours(f.shape, centre)) == (14 if f.ndim == 3 else 6)


def _elder_pairs(shape, key):
    """0-dimensional superlevel-set persistence pairs by the elder rule: sweep
    the vertices from the largest key down with a union-find of the swept
    ones; where components meet, every one but the component of the largest
    maximum dies, paired with the meeting vertex.  {maximum: saddle}; the
    global maximum stays unpaired."""
    parent, top, pairs = {}, {}, {}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for v in np.argsort(-key, kind="stable"):
        v = int(v)
        roots = {find(u) for u in lts.neighbours(shape, v) if u in parent}
        parent[v] = v
        if not roots:
            top[v] = v
            continue
        best = max(roots, key=lambda r: key[top[r]])
        for r in roots:
            if r != best:
                pairs[top[r]] = v
            parent[r] = best
        parent[v] = best
    return pairs


def _merged_fields():
    yield fieldgen.gaussian_field((12, 10, 9), 4, 5, noise=("uniform", 2e-2))
    yield fieldgen.iid_field((8, 7, 6), 13)
    yield fieldgen.tie_field((8, 9, 6), 6, 3)
    yield fieldgen.gaussian_field((30, 26), 7, 4, noise=("uniform", 5e-2))


@pytest.mark.parametrize("maxima", [True, False])
def test_merged_removes_exactly_the_elder_pairs_within_epsilon(maxima):
    """Merged propagations from every maximum (minimum), budgets unbounded:
    an extremum is removed, at saddle s, exactly when the elder rule pairs
    it with s and the value difference is at most epsilon; every other one
    is persistent; a removed extremum's component is the strict superlevel
    component of s plus s.  The independent propagations differ on some
    extrema (the elder one at a saddle), so the merging is exercised."""
    differs = 0
    for f in _merged_fields():
        fv = f.ravel()
        rank, _ = order_field(f)
        key = rank.astype(np.int64) if maxima else rank.size - 1 - rank.astype(np.int64)
        mn, mx = extrema(oracle.classify(f).codes)
        ext = mx if maxima else mn
        pairs = _elder_pairs(f.shape, key)
        assert set(pairs) | {int(np.argmax(key))} == set(int(m) for m in ext)
        big = f.size + 1
        for eps in (0.0, 0.01, 0.05, 0.3, np.inf):
            st, sd, vi = lts.propagate_merged(f, ext, eps, maxima, big, big, rank=rank)
            for i, m in enumerate(ext):
                m = int(m)
                s = pairs.get(m)
                d = None if s is None else (np.float32(fv[m] - fv[s]) if maxima else
                                            np.float32(fv[s] - fv[m]))
                if s is not None and d <= np.float32(eps):
                    assert (st[i], sd[i]) == (lts.SADDLE, s), (m, eps)
                    comp = lts.superlevel_component(f.shape, key, m, key[s] + 1)
                    assert vi[i] == len(comp) + 1
                else:
                    assert (st[i], sd[i]) == (lts.PERSISTENT, -1), (m, eps)
            ind = lts.propagate_all(f, ext, eps, maxima, big, big, rank=rank)
            differs += int(np.count_nonzero(ind[0] != st))
    assert differs > 0


def test_merged_result_does_not_depend_on_arrival_order():
    """Budgets small enough to stop some merges: any order of starting the
    propagations gives the same statuses, saddles and counts."""
    f = fieldgen.gaussian_field((14, 12, 10), 9, 4, noise=("uniform", 3e-2))
    _, mx = extrema(oracle.classify(f).codes)
    rng = np.random.default_rng(5)
    for mv, mf, eps in ((8, 40, 0.05), (32, 128, 0.1), (16, 64, np.inf)):
        ref = lts.propagate_merged(f, mx, eps, True, mv, mf)
        assert np.count_nonzero(ref[0] == lts.SADDLE) > 0
        for _ in range(3):
            got = lts.propagate_merged(f, mx, eps, True, mv, mf, order=rng.permutation(len(mx)))
            for a, b in zip(ref, got):
                assert np.array_equal(a, b)


def test_merged_two_bumps_and_chain_closed_form():
    """2D profiles along x, constant bands in y with a small slope towards
    the middle row.  Two peaks joined at a pass: with epsilon at or above
    the lower peak's height over the pass it is removed there and the higher
    one is persistent (with no epsilon its propagation takes the whole grid).  Three peaks
    (1.0, 2.0, 1.5) with passes 0.6 and 0.9: the peak 1.5 first merges into
    the peak 2.0's component at the pass 0.9; with epsilon 0.7 both lower
    peaks go and the merged propagation, led by 2.0, stops as persistent."""
    ny, cy = 7, 3
    y = np.arange(ny)[:, None]

    def grid(g):
        return (np.asarray(g, np.float32)[None, :] - 0.01 * np.abs(y - cy)).astype(np.float32)

    f = grid([0, 0.5, 1, 0.7, 0.6, 0.5, 1.2, 1.6, 2, 1.5, 1])
    big = f.size + 1
    pk = [cy * 11 + 2, cy * 11 + 8]
    st, sd, vi = lts.propagate_merged(f, pk, 0.5, True, big, big)
    assert list(st) == [lts.SADDLE, lts.PERSISTENT] and sd[0] == cy * 11 + 5
    st, sd, vi = lts.propagate_merged(f, pk, np.inf, True, big, big)
    assert list(st) == [lts.SADDLE, lts.PERSISTENT] and list(vi) == [22, f.size]
    st, sd, _ = lts.propagate_merged(f, pk, 0.49, True, big, big)
    assert list(st) == [lts.PERSISTENT, lts.PERSISTENT]

    g = [0, 1.0, 0.6, 2.0, 0.9, 1.5, 0.2]
    f = grid(g)
    n = len(g)
    pk = [cy * n + 1, cy * n + 3, cy * n + 5]
    st, sd, _ = lts.propagate_merged(f, pk, 0.7, True, big, big)
    assert list(st) == [lts.SADDLE, lts.PERSISTENT, lts.SADDLE]
    assert list(sd) == [cy * n + 2, -1, cy * n + 4]
    # epsilon 0.45: the peak 1.0 goes (0.4), 1.5 stays (0.6)
    st, sd, _ = lts.propagate_merged(f, pk, 0.45, True, big, big)
    assert list(st) == [lts.SADDLE, lts.PERSISTENT, lts.PERSISTENT]


def test_merged_invalid_entries():
    f = fieldgen.iid_field((9, 8, 7), 3)
    _, mx = extrema(oracle.classify(f).codes)
    notmax = next(v for v in range(f.size) if v not in set(mx.tolist()))
    st, sd, vi = lts.propagate_merged(f, [int(mx[0]), f.size, notmax, int(mx[1])], 0.1)
    assert list(st[1:3]) == [lts.INVALID, lts.INVALID] and list(sd[1:3]) == [-1, -1]
    assert list(vi[1:3]) == [0, 0]


def test_merged_budget_at_a_merge():
    """The budget reading at a merge, on the two-peak profile: the higher
    peak reaches the pass with 36 vertices, the lower one with 22, so their
    union holds 57.  With max_visited 57 the union itself is over budget
    (the merge ends it, visited 57); with 58 the merged propagation takes
    one more vertex before the budget stops it; with 35 the higher peak
    never reaches the pass."""
    ny, cy = 7, 3
    y = np.arange(ny)[:, None]
    g = np.array([0, 0.5, 1, 0.7, 0.6, 0.5, 1.2, 1.6, 2, 1.5, 1], np.float32)
    f = (g[None, :] - 0.01 * np.abs(y - cy)).astype(np.float32)
    pk = [cy * 11 + 2, cy * 11 + 8]
    rank, _ = order_field(f)
    pass_v = cy * 11 + 5
    comp_hi = lts.superlevel_component(f.shape, rank.astype(np.int64), pk[1], int(rank[pass_v]) + 1)
    comp_lo = lts.superlevel_component(f.shape, rank.astype(np.int64), pk[0], int(rank[pass_v]) + 1)
    assert (len(comp_hi) + 1, len(comp_lo) + 1) == (36, 22)
    for mv, visited_hi in ((57, 57), (58, 58), (36, 57), (35, 35)):
        st, sd, vi = lts.propagate_merged(f, pk, np.inf, True, mv, 1000)
        assert list(st) == [lts.SADDLE, lts.BUDGET] and sd[0] == pass_v, mv
        assert list(vi) == [22, visited_hi], mv
