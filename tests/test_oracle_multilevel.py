"""Pins of the oracle's multi-level high-frequency path (Algorithm 1 with more
than one HF level): HF-M2M and HF-L2L between HF widths through the wedge
hierarchy of Figure 2, the closure of the needed (box, wedge) slots across
levels, the skeletons of Eq. 2 at widths 2 and 4 (with the parent check-point
augmentation), the offsets an interaction list can hold beyond w = 1, and the
Morton order of the octree (Section 2.2).

The tree is a sphere of diameter K = 8 (N = 8,192), whose interaction lists
are non-empty at w = 2 and w = 1, so the pass runs M2M from w = 1 up to w = 2
and L2L from w = 2 down to w = 1 (the K = 4 sphere of the other oracle pins
has one HF level only).  Each planted mistake below is one that a plausible
slip in the oracle would make; a pin must fail on it.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import fmm as F
from oracle import operators as O
from oracle import tree as T
from oracle.kernel import direct_sum, rel_l2
from paper_1311_4257_amd import workloads
from tests.helpers import oracle_opset

TAU = 1e-4      # the multi-level accuracy pins
TAU_FAST = 1e-3  # symmetry, linearity and planted mistakes (smaller ranks, faster)


@pytest.fixture(scope="module")
def case8():
    pts = workloads.sphere_points(8192, 8.0, seed=8)
    f = workloads.densities(8192, 1, seed=108)
    st = T.build_structure(pts, 8.0)
    return pts, f, st, direct_sum(pts, f)


def test_tree_has_two_hf_levels(case8):
    _, _, st, _ = case8
    assert st.w_top == 2
    widths = [int(st.tree.width(l)) for l in st.hf_levels]
    assert widths == [2, 1]
    assert all(len(st.lists[l].tgt) > 0 for l in st.hf_levels)


def test_multilevel_pass_matches_direct_sum(case8):
    """The whole pass (S2M, M2M 1 -> 2, M2L at w = 2 and 1, L2L 2 -> 1 -> LF, LF-M2L,
    L2T, near field) against Eq. 1 on every target.  Each translation carries the
    skeleton truncation tau of Eq. 2, so the error is a small multiple of tau;
    looser skeletons give a larger error."""
    pts, f, st, ref = case8
    err = rel_l2(F.fmm_apply(st, oracle_opset(TAU, 2), f), ref)
    assert err < 5 * TAU, err
    err_loose = rel_l2(F.fmm_apply(st, oracle_opset(TAU_FAST, 2), f), ref)
    assert err < err_loose < 5 * TAU_FAST, (err, err_loose)


def test_multilevel_operator_is_complex_symmetric(case8):
    """G(x, y) = G(y, x): with L2L = M2M^T at every width (w = 2 -> 1 included) and
    reciprocal M2L, g^T A f = f^T A g to rounding."""
    pts, f, st, _ = case8
    ops = oracle_opset(TAU_FAST, 2)
    g = workloads.densities(len(pts), 1, seed=109)[0]
    a = g @ F.fmm_apply(st, ops, f[0])
    b = f[0] @ F.fmm_apply(st, ops, g)
    assert abs(a - b) < 1e-11 * abs(a)


def test_needed_slots_close_under_the_hierarchy(case8):
    """Every pair's source (A, l_out) is an outgoing slot and its target (B, l_in)
    an incoming slot of its level; every needed slot of a box at width 2w has its
    children's slots at the mapped wedge (f, i // 2, j // 2) at width w (HF-M2M
    reads them, HF-L2L writes them); and no slot is needed for any other reason
    (the closure is exact, not a superset)."""
    _, _, st, _ = case8
    tr = st.tree
    checked = 0
    for l in st.out_slots:
        w = int(tr.width(l))
        outs = set(map(tuple, st.out_slots[l].tolist()))
        ins = set(map(tuple, st.in_slots[l].tolist()))
        pl = st.lists[l]
        used_out = set(zip(pl.src.tolist(), pl.dir_out.tolist()))
        used_in = set(zip(pl.tgt.tolist(), pl.dir_in.tolist()))
        assert used_out <= outs and used_in <= ins, l
        # slots demanded from the parent level
        dem_out, dem_in = set(), set()
        if l - 1 in st.out_slots:
            kids = T.children(tr, l - 1)
            for (p, d) in st.out_slots[l - 1].tolist():
                dem_out.update((c, T.direction_down(d, 2 * w)) for c in kids[p])
            for (p, d) in st.in_slots[l - 1].tolist():
                dem_in.update((c, T.direction_down(d, 2 * w)) for c in kids[p])
        assert outs == used_out | dem_out and ins == used_in | dem_in, l
        if l + 1 in st.out_slots:
            kids = T.children(tr, l)
            fine_out = set(map(tuple, st.out_slots[l + 1].tolist()))
            fine_in = set(map(tuple, st.in_slots[l + 1].tolist()))
            for (b, d) in outs:
                for c in kids[b]:
                    assert (c, T.direction_down(d, w)) in fine_out
                    checked += 1
            for (b, d) in ins:
                for c in kids[b]:
                    assert (c, T.direction_down(d, w)) in fine_in
                    checked += 1
    assert checked > 1000  # the w = 2 -> w = 1 closure is exercised


def test_morton_keys_by_hand():
    """Octant o = x_bit | y_bit << 1 | z_bit << 2 per level, root octant most
    significant (Section 2.2's level-by-level subdivision)."""
    ix = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1],
                   [2, 0, 0], [3, 1, 0], [0, 2, 3], [3, 3, 3]])
    # D = 2: key = 8 * octant(level 1) + octant(level 2)
    want = [1, 2, 4, 7, 8, 8 + 3, 8 * 6 + 4 + 0, 63]
    assert T.morton(ix, 2).tolist() == want
    # K = 8, D = 4: coordinate -2.25 is leaf 3 = 0011b, +2.25 is leaf 12 = 1100b.
    # (-2.25, -2.25, -2.25): octants 0, 0, 7, 7 -> key 63
    # (+2.25, -2.25, -2.25): octants 1, 1, 6, 6 -> key ((1 * 8 + 1) * 8 + 6) * 8 + 6 = 630
    # (-2.25, +2.25, -2.25): octants 2, 2, 5, 5 -> 1197;  (-2.25, -2.25, +2.25): 4, 4, 3, 3 -> 2331
    pts = np.array([[-2.25, -2.25, -2.25], [2.25, -2.25, -2.25], [-2.25, 2.25, -2.25], [-2.25, -2.25, 2.25]])
    tr = T.build_tree(pts, 8.0)
    assert tr.D == 4
    assert tr.levels[4].keys.tolist() == [63, 630, 1197, 2331]
    assert tr.levels[1].keys.tolist() == [0, 1, 2, 4]     # the level-l box: key >> 3 (D - l)


@pytest.mark.parametrize("w", [1, 2, 4])
def test_region_offsets_are_exactly_the_possible_list_offsets(w):
    """An interaction pair at width w joins boxes whose parents are near at 2w
    (children of N^P) and that are not near at w (Section 2.2): brute force over
    every child position and every parent offset in the near field at 2w."""
    want = set()
    lim2 = T.near_limit4(2 * w)
    r = 2
    while 4 * (2 * (r + 1) - 1) ** 2 <= lim2:
        r += 1
    for m in itertools.product(range(-r, r + 1), repeat=3):
        if 4 * T.near_sum(np.array(m)) > lim2:
            continue
        for o in itertools.product((0, 1), repeat=3):        # child position of B in its parent
            for q in itertools.product((0, 1), repeat=3):    # child position of A in its parent
                n = tuple(2 * mk + qk - ok for mk, qk, ok in zip(m, q, o))
                if not T.is_near(np.array(n), w):
                    want.add(n)
    got = set(map(tuple, O.region_offsets(float(w)).tolist()))
    assert got == want


def test_list_offsets_lie_in_the_regions(case8):
    """Every offset of the K = 8 tree's lists is in region_offsets of its width, and
    its wedge is the wedge the skeleton of that region serves."""
    _, _, st, _ = case8
    for l in st.hf_levels:
        w = int(st.tree.width(l))
        reg = set(map(tuple, O.region_offsets(float(w)).tolist()))
        pl = st.lists[l]
        for n, di in zip(pl.offset.tolist(), pl.dir_in.tolist()):
            assert tuple(n) in reg
            assert T.direction(n, w) == di


def _heldout(sk, w, d, rng):
    offs = O.region_offsets(float(w))
    dirs = np.array([T.direction(n, w) for n in offs.tolist()])
    X = O._sample_boxes(rng, offs[dirs == d] * float(w), float(w), 800)
    Y = (rng.random((300, 3)) - 0.5) * w
    return O.heldout_error(sk, X, Y)


def test_skeletons_heldout_at_width_2():
    """Eq. 2 on fresh far-region and box samples at w = 2, every wedge."""
    ops = oracle_opset(TAU, 2)
    rng = np.random.default_rng(202)
    for d, sk in enumerate(ops.hf[2]):
        assert _heldout(sk, 2, d, rng) < 10 * TAU, d


def test_skeletons_heldout_at_width_4():
    """Eq. 2 at w = 4 on a spread of wedges (all six faces)."""
    ops = oracle_opset(TAU_FAST, 4)
    rng = np.random.default_rng(404)
    for d in range(0, 96, 7):
        assert _heldout(ops.hf[4][d], 4, d, rng) < 10 * TAU_FAST, d


def test_child_skeletons_reproduce_the_parent_check_points():
    """The parent augmentation: a w = 1 skeleton must also represent G at the
    check points of every w = 2 wedge that maps to it, seen from each of the 8
    child positions (this is where HF-M2M evaluates it)."""
    ops = oracle_opset(TAU, 2)
    rng = np.random.default_rng(7)
    dl = O.child_deltas(1.0)
    for lp, sp in enumerate(ops.hf[2]):
        d = T.direction_down(lp, 2)
        sk = ops.hf[1][d]
        X = (sp.a[None, :, :] - dl[:, None, :]).reshape(-1, 3)
        Y = rng.random((200, 3)) - 0.5
        assert O.heldout_error(sk, X, Y) < 10 * TAU, lp


# --------------------------------------------------------------------------
# planted mistakes at w >= 2
# --------------------------------------------------------------------------

def test_planted_wrong_wedge_hierarchy_breaks_the_pass(case8, monkeypatch):
    """HF-M2M / HF-L2L mapping a wedge to the child wedge on the opposite face
    (a sign slip in the face index 2 a + [n_a < 0])."""
    pts, f, st, ref = case8
    ops = oracle_opset(TAU_FAST, 2)
    good = rel_l2(F.fmm_apply(st, ops, f), ref)

    def flipped(l, w2):
        w = w2 // 2
        face, rem = divmod(l, w2 * w2)
        i, j = divmod(rem, w2)
        return ((face ^ 1) * w + i // 2) * w + j // 2

    monkeypatch.setattr(F, "direction_down", flipped)
    try:
        bad = rel_l2(F.fmm_apply(st, ops, f), ref)
    except KeyError:
        bad = np.inf                          # a slot the wrong map asks for does not exist
    assert bad > 10 * good, (good, bad)


def _parent_point_errors(ops) -> np.ndarray:
    """Eq. 2 error of each w = 1 skeleton at the check points of the w = 2 wedges
    that map to it, seen from the 8 child positions (where HF-M2M evaluates it)."""
    rng = np.random.default_rng(7)
    dl = O.child_deltas(1.0)
    errs = []
    for lp, sp in enumerate(ops.hf[2]):
        X = (sp.a[None, :, :] - dl[:, None, :]).reshape(-1, 3)
        Y = rng.random((200, 3)) - 0.5
        errs.append(O.heldout_error(ops.hf[1][T.direction_down(lp, 2)], X, Y))
    return np.array(errs)


def test_planted_missing_parent_augmentation_breaks_the_pass(monkeypatch):
    """Skeletons built without the parent wedges' check points: a w = 1 skeleton
    then reproduces G at those points several times worse than the augmented
    one.  (The end-to-end pass moves much less: the M2M / L2L hops are a small
    part of its error at this tau.)"""
    eg = _parent_point_errors(oracle_opset(TAU_FAST, 2))
    monkeypatch.setattr(O, "direction_down", lambda l, w2: -1)
    bad = O.build_opset(TAU_FAST, 2)
    monkeypatch.undo()
    eb = _parent_point_errors(bad)
    assert np.median(eb) > 2 * np.median(eg) and eb.max() > 2 * eg.max(), (eg.max(), eb.max())
