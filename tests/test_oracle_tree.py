"""Pins of the oracle's octree, near fields, lists and wedges (Section 2.2)
against brute force, exact geometry and the paper's Proposition 1."""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

from oracle import tree as T
from paper_1311_4257_amd import workloads


@pytest.fixture(scope="module")
def st4():
    pts, _, cfg = workloads.make_config("sphere4")
    return T.build_structure(pts, cfg["K"])


def test_leaf_coordinates_brute_force():
    K = 4.0
    rng = np.random.default_rng(0)
    pts = rng.uniform(-K / 2, K / 2, size=(500, 3)) / math.sqrt(3)
    # points exactly on box faces (interior faces go up, the upper boundary is clamped)
    pts[:8] = [[-2, 0, 0], [2, 0, 0], [0, -2, 0], [0.5, 0.5, 0.5], [-0.5, 0, 1.0],
               [0, 0, 0], [1.5, -1.5, 0.25], [0, 0, 2]]
    D = 3
    ix = T.leaf_coords(pts, K, D)
    edges = -K / 2 + 0.5 * np.arange(2 ** D + 1)      # exact dyadic edges
    for p, c in zip(pts, ix):
        for k in range(3):
            want = int(np.sum(edges[1:-1] <= p[k]))   # number of interior edges at or below x
            assert c[k] == want


def test_morton_order_and_level_tables(st4):
    tr = st4.tree
    D = tr.D
    ix = T.leaf_coords(tr.points, tr.K, D)
    key = T.morton(ix, D)
    assert np.all(np.diff(key) >= 0)
    # ties broken by original index
    same = np.diff(key) == 0
    assert np.all(np.diff(tr.perm)[same] > 0)
    for l in range(D + 1):
        lv = tr.levels[l]
        for b in range(len(lv.coords)):
            c = ix[lv.start[b]:lv.end[b]] >> (D - l)
            assert np.all(c == lv.coords[b])
        assert lv.end[-1] == len(tr.points)
        if l > 0:
            up = tr.levels[l - 1]
            assert np.all(up.coords[lv.parent] == lv.coords >> 1)


def test_near_field_integer_test_equals_geometry():
    """A in N^B iff box A meets the closed ball about c_B of radius max(sqrt3 w/2, 3 w^2/4)."""
    for w in [0.5, 1.0, 2.0, 4.0, 8.0]:
        R2 = max(3 * w * w / 4, 9 * w ** 4 / 16)
        r = int(math.ceil(max(math.sqrt(3) / 2, 3 * w / 4) + 1))
        for n in itertools.product(range(-r, r + 1), repeat=3):
            # squared distance from c_B to box A (exact: dyadic values)
            d2 = sum(max(0.0, abs(k) * w - w / 2) ** 2 for k in n)
            assert (d2 <= R2) == bool(T.is_near(np.array(n), w)), (w, n)


def test_covering_each_leaf_pair_exactly_once(st4):
    """Every ordered pair of distinct leaves is handled by the near-field sum or by
    exactly one interaction list on exactly one level."""
    tr = st4.tree
    D = tr.D
    nleaf = len(tr.levels[D].coords)
    count = np.zeros((nleaf, nleaf), dtype=np.int64)
    nb = st4.near
    count[nb.tgt, nb.src] += 1
    # ancestors of each leaf per level
    anc = {D: np.arange(nleaf)}
    for l in range(D, 0, -1):
        anc[l - 1] = tr.levels[l].parent[anc[l]]
    for l, pl in st4.lists.items():
        if not len(pl.tgt):
            continue
        pairs = set(zip(pl.tgt.tolist(), pl.src.tolist()))
        A = anc[l]
        hit = np.array([[(A[i], A[j]) in pairs for j in range(nleaf)] for i in range(nleaf)])
        count += hit
    assert np.all(count == 1)        # the diagonal: each leaf's own near-field block


def test_lists_symmetric_with_swapped_wedges(st4):
    for l, pl in st4.lists.items():
        fwd = {(b, a): (di, do) for b, a, di, do in zip(pl.tgt.tolist(), pl.src.tolist(),
                                                        pl.dir_in.tolist(), pl.dir_out.tolist())}
        for (b, a), (di, do) in fwd.items():
            assert (a, b) in fwd
            assert fwd[(a, b)] == (do, di)


@pytest.mark.parametrize("K,kind", [(4.0, "sphere"), (8.0, "sphere"), (16.0, "ellipsoid")])
def test_proposition1_empty_lists_at_the_top(K, kind):
    """Proposition 1: for w >= sqrt(4K/3 + 1/3) + sqrt(1/3) the near field holds every box."""
    if kind == "sphere":
        pts = workloads.sphere_points(3000, K, seed=3)
    else:
        pts = workloads.ellipsoid_points(3000, (K / 2, K / 4, K / 8), seed=3)
    st = T.build_structure(pts, K)
    bound = math.sqrt(4 * K / 3 + 1 / 3) + math.sqrt(1 / 3)
    for l, pl in st.lists.items():
        if st.tree.width(l) >= bound:
            assert len(pl.tgt) == 0, (K, l)
    assert st.w_top < 2 * math.sqrt(K)


def test_direction_against_float_reference():
    """Face = axis of largest |n_k| and sign; cell = floor of the tangent-plane coordinate."""
    rng = np.random.default_rng(1)
    for w in [1, 2, 4, 8]:
        for _ in range(3000):
            n = rng.integers(-40, 41, size=3)
            if not n.any():
                continue
            m = np.max(np.abs(n))
            if np.sum(np.abs(n) == m) > 1:
                continue                      # face ties are pinned separately
            a = int(np.argmax(np.abs(n)))
            face = 2 * a + (n[a] < 0)
            cells = []
            tie = False
            for t in range(3):
                if t == a:
                    continue
                x = (n[t] / m + 1) / 2 * w    # in [0, w]
                if abs(x - round(x)) < 1e-12:
                    tie = True
                cells.append(min(int(math.floor(x)), w - 1))
            if tie:
                continue
            want = (face * w + cells[0]) * w + cells[1]
            assert T.direction(n, w) == want


def test_direction_ties_go_first():
    # face ties -> smallest axis; cell boundaries -> lower cell
    assert T.direction([3, 3, 0], 1) == 0          # x and y tie: face +x
    assert T.direction([-3, 3, 3], 1) == 1         # all tie: face -x
    # on the central boundary (n_t = 0) of a 2-cell face the lower cell is taken
    assert T.direction([5, 0, 0], 2) == 0
    assert T.direction([5, 1, 0], 2) == 2          # y cell 1, z cell 0
    assert T.direction([0, 0, -7], 2) == 5 * 4     # face -z, cells (0, 0)


def test_direction_hierarchy_is_exact():
    """A wedge at width 2w lies inside wedge (f, i//2, j//2) at width w (Figure 2)."""
    for w in [1, 2, 4]:
        r = 12
        for n in itertools.product(range(-r, r + 1), repeat=3):
            if n == (0, 0, 0):
                continue
            assert T.direction_down(T.direction(n, 2 * w), 2 * w) == T.direction(n, w)


def test_needed_slots_close_under_hierarchy(st4):
    tr = st4.tree
    for l, slots in st4.out_slots.items():
        if l + 1 >= tr.D:
            continue
        kids = T.children(tr, l)
        w = int(tr.width(l))
        fine = set(map(tuple, st4.out_slots[l + 1].tolist()))
        for b, d in slots.tolist():
            for c in kids[b]:
                assert (c, T.direction_down(d, w)) in fine
