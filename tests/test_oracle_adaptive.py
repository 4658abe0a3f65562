"""Pins of the oracle's adaptive low-frequency tree (Section 2.2: the octree is
non-adaptive in the high-frequency regime and adaptive in the low-frequency
regime, where a box splits while it holds more than a fixed number of points)
and of the pass over it (Algorithm 1's LF-M2M postorder loop and its
LF-M2L / LF-L2L preorder loop, with the near field between leaves of
different sizes).

The point set is a dense K = 4 sphere (N = 12,000), so boxes of width 1/2
hold ~45 points and split down to width 1/8 or 1/16 for leaf_max = 16.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import fmm as F
from oracle import operators as O
from oracle import tree as T
from oracle.adaptive import deep_lf_skeletons, lf_skeleton
from oracle.kernel import direct_sum, rel_l2
from paper_1311_4257_amd import workloads
from tests.helpers import oracle_opset

TAU = 1e-4
LEAF_MAX = 16
EXTRA = 3


@pytest.fixture(scope="module")
def case():
    pts = workloads.sphere_points(12000, 4.0, seed=41)
    f = workloads.densities(len(pts), 1, seed=42)[0]
    st = T.build_structure(pts, 4.0, leaf_max=LEAF_MAX, extra=EXTRA)
    ops = oracle_opset(TAU, 1)
    deep = deep_lf_skeletons(ops, st.tree.Dmax - st.tree.D)
    tg = np.arange(0, len(pts), 5)
    return pts, f, st, ops, deep, tg, direct_sum(pts, f, tg)


def test_adaptive_split_rule(case):
    """Width >= 1 boxes always split, width-1 boxes into width 1/2; a box of width
    <= 1/2 is split exactly when it holds more than leaf_max points and is above
    the deepest level; its children are its non-empty octants, and each box
    holds exactly the points whose finest-level cell lies in it."""
    pts, _, st, _, _, _, _ = case
    tr = st.tree
    assert tr.Dmax > tr.D + 1                        # several low-frequency levels
    Dm = tr.D + EXTRA
    ix = T.leaf_coords(tr.points, tr.K, Dm)
    for l, lv in enumerate(tr.levels):
        n = lv.end - lv.start
        if l < tr.D:
            assert not lv.leaf.any()
        elif l < Dm:
            assert np.array_equal(~lv.leaf, n > LEAF_MAX), l
        for b in range(len(lv.coords)):
            assert np.all(ix[lv.start[b]:lv.end[b]] >> (Dm - l) == lv.coords[b])
        if l + 1 < len(tr.levels):
            kids = T.children(tr, l)
            for b in range(len(lv.coords)):
                if lv.leaf[b]:
                    assert kids[b] == []
                else:
                    cs = tr.levels[l + 1].coords[kids[b]]
                    assert np.all(cs >> 1 == lv.coords[b])
                    assert tr.levels[l + 1].start[kids[b][0]] == lv.start[b]
                    assert tr.levels[l + 1].end[kids[b][-1]] == lv.end[b]
    # every point is in exactly one leaf
    cover = np.zeros(len(pts), dtype=np.int64)
    for l, b in tr.leaf_boxes():
        cover[tr.levels[l].start[b]:tr.levels[l].end[b]] += 1
    assert np.all(cover == 1)


def test_covering_each_leaf_pair_exactly_once(case):
    """Every ordered pair of leaves (of any sizes) is handled exactly once: by the
    near field or by one interaction-list pair of their ancestors on one level."""
    _, _, st, _, _, _, _ = case
    tr = st.tree
    leaves = tr.leaf_boxes()
    idx = {lb: i for i, lb in enumerate(leaves)}
    cnt = np.zeros((len(leaves), len(leaves)), dtype=np.int32)
    for B, A in st.near:
        cnt[idx[B], idx[A]] += 1
    memo = {}

    def under(l, b):  # leaf indices below box b of level l
        if (l, b) not in memo:
            if tr.levels[l].leaf[b]:
                memo[(l, b)] = [idx[(l, b)]]
            else:
                memo[(l, b)] = [i for c in T.children(tr, l)[b] for i in under(l + 1, c)]
        return memo[(l, b)]

    for l, pl in st.lists.items():
        for B, A in zip(pl.tgt.tolist(), pl.src.tolist()):
            cnt[np.ix_(under(l, B), under(l, A))] += 1
    assert cnt.min() == 1 and cnt.max() == 1


def test_near_lists_are_symmetric(case):
    _, _, st, _, _, _, _ = case
    pairs = set(st.near)
    assert all((A, B) in pairs for B, A in pairs)
    # coarse-fine pairs (sizes differ) are present: the adaptive part of the near field
    assert any(B[0] != A[0] for B, A in pairs)


def test_deep_skeletons_heldout(case):
    """Eq. 2 at widths 1/4 and 1/8 on fresh samples of the interaction-list region."""
    _, _, _, ops, deep, _, _ = case
    rng = np.random.default_rng(5)
    w = 0.25
    for sk in deep[:2]:
        X = O._sample_boxes(rng, O.region_offsets(w) * w, w, 600)
        Y = (rng.random((300, 3)) - 0.5) * w
        assert O.heldout_error(sk, X, Y) < 10 * TAU, w
        w /= 2
    assert lf_skeleton(ops, deep, 0.5) is ops.lf and lf_skeleton(ops, deep, 0.125) is deep[1]


def test_adaptive_pass_matches_direct_sum(case):
    pts, f, st, ops, deep, tg, ref = case
    err = rel_l2(F.fmm_apply(st, ops, f, deep=deep)[tg], ref)
    assert err < 5 * TAU, err


def test_adaptive_operator_is_complex_symmetric(case):
    """LF-L2L = LF-M2M^T and symmetric near lists: g^T A f = f^T A g to rounding."""
    pts, f, st, ops, deep, _, _ = case
    g = workloads.densities(len(pts), 1, seed=43)[0]
    a = g @ F.fmm_apply(st, ops, f, deep=deep)
    b = f @ F.fmm_apply(st, ops, g, deep=deep)
    assert abs(a - b) < 1e-11 * abs(a)


def test_no_split_reduces_to_the_uniform_pass():
    """leaf_max above every box's count: the adaptive tree is the uniform one (the
    points are only ordered by a finer key), and the pass gives the same result
    to rounding."""
    pts, f, cfg = workloads.make_config("sphere4")
    ops = oracle_opset(1e-3, 1)
    st_u = T.build_structure(pts, 4.0)
    st_a = T.build_structure(pts, 4.0, leaf_max=10 ** 6, extra=2)
    assert st_a.tree.Dmax == st_a.tree.D
    for l in range(st_u.tree.D + 1):
        assert np.array_equal(st_u.tree.levels[l].coords, st_a.tree.levels[l].coords)
    assert rel_l2(F.fmm_apply(st_a, ops, f), F.fmm_apply(st_u, ops, f)) < 1e-13


def test_planted_same_level_near_field_breaks_the_pass(case, monkeypatch):
    """A near field with only the adjacent leaves of the same size (the uniform
    rule) misses the coarse-fine pairs."""
    pts, f, st, ops, deep, tg, ref = case
    same = [(B, A) for B, A in st.near if B[0] == A[0]]
    st2 = T.Structure(tree=st.tree, lists=st.lists, near=same, hf_levels=st.hf_levels,
                      out_slots=st.out_slots, in_slots=st.in_slots)
    good = rel_l2(F.fmm_apply(st, ops, f, deep=deep)[tg], ref)
    bad = rel_l2(F.fmm_apply(st2, ops, f, deep=deep)[tg], ref)
    assert bad > 100 * good, (good, bad)


def test_planted_wrong_width_skeleton_breaks_the_pass(case):
    """Every deeper LF level using the width-1/2 skeleton (a width mix-up in
    LF-M2M / LF-L2L / LF-M2L)."""
    pts, f, st, ops, deep, tg, ref = case
    good = rel_l2(F.fmm_apply(st, ops, f, deep=deep)[tg], ref)
    bad = rel_l2(F.fmm_apply(st, ops, f, deep=[ops.lf] * len(deep))[tg], ref)
    assert bad > 10 * good, (good, bad)
