"""Pins of the oracle's skeletons (Eq. 2) and evaluation pass (Algorithm 1)
against the direct sum of Eq. 1, the held-out error of Eq. 2, reciprocity and
special cases.  A planted mistake in the oracle must break a pin."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import fmm as F
from oracle import operators as O
from oracle.kernel import direct_sum, green, rel_l2
from oracle.tree import build_structure
from paper_1311_4257_amd import workloads
from tests.helpers import oracle_opset


@pytest.fixture(scope="module")
def case4():
    pts, f, cfg = workloads.make_config("sphere4")
    st = build_structure(pts, cfg["K"])
    return pts, f, st, direct_sum(pts, f)


def test_skeleton_heldout_error_within_tau():
    """Eq. 2 on fresh points of the same far region and box: error of order tau."""
    tau = 1e-4
    ops = oracle_opset(tau, 1)
    rng = np.random.default_rng(42)
    offs = O.region_offsets(1.0)
    dirs = np.array([O.direction(n, 1) for n in offs.tolist()])
    for d, sk in enumerate(ops.hf[1]):
        X = O._sample_boxes(rng, offs[dirs == d] * 1.0, 1.0, 600)
        Y = (rng.random((300, 3)) - 0.5)
        assert O.heldout_error(sk, X, Y) < 10 * tau, d
    X = O._sample_boxes(rng, O.region_offsets(0.5) * 0.5, 0.5, 600)
    Y = (rng.random((300, 3)) - 0.5) * 0.5
    assert O.heldout_error(ops.lf, X, Y) < 10 * tau


def test_ranks_grow_with_accuracy_like_table1():
    """Table 1: the separation rank grows as the target accuracy tightens (1e-4 -> 1e-6
    multiplies it by about 1.6-1.8); here tau 1e-3 -> 1e-4."""
    lo, hi = oracle_opset(1e-3, 1), oracle_opset(1e-4, 1)
    assert hi.rank(1) > lo.rank(1) and hi.lf.r > lo.lf.r
    assert 1.2 < hi.rank(1) / lo.rank(1) < 1.8


def test_fmm_matches_direct_sum(case4):
    pts, f, st, ref = case4
    ops = oracle_opset(1e-4, 1)
    u = F.fmm_apply(st, ops, f)
    err = rel_l2(u, ref)
    assert err < 3e-4, err                       # per-skeleton tau = 1e-4
    ops2 = oracle_opset(1e-3, 1)
    err2 = rel_l2(F.fmm_apply(st, ops2, f), ref)
    assert err < err2 < 3e-3                     # looser skeletons, larger error


def test_fmm_operator_is_complex_symmetric(case4):
    """G(x, y) = G(y, x): M2L is reciprocal, L2L = M2M^T and L2T = S2M^T, so
    g^T A_fmm f = f^T A_fmm g up to rounding."""
    pts, f, st, _ = case4
    ops = oracle_opset(1e-3, 1)
    g = workloads.densities(len(pts), 1, seed=77)[0]
    a = g @ F.fmm_apply(st, ops, f[0])
    b = f[0] @ F.fmm_apply(st, ops, g)
    assert abs(a - b) < 1e-11 * abs(a)


def test_fmm_is_linear(case4):
    pts, f, st, _ = case4
    ops = oracle_opset(1e-3, 1)
    G2 = workloads.densities(len(pts), 2, seed=78)
    u = F.fmm_apply(st, ops, G2)
    v = F.fmm_apply(st, ops, (1 - 2j) * G2[0] + 3 * G2[1])
    assert rel_l2(v, (1 - 2j) * u[0] + 3 * u[1]) < 1e-12


def test_two_adjacent_leaves_reduce_to_direct_sum():
    """All points in two adjacent leaves: no far field, the pass is the direct sum."""
    rng = np.random.default_rng(9)
    pts = np.concatenate([rng.uniform(0.01, 0.49, (30, 3)), rng.uniform(0.01, 0.49, (30, 3)) + [0.5, 0, 0]])
    f = workloads.densities(60, 1, seed=10)[0]
    st = build_structure(pts, 4.0)
    assert all(len(pl.tgt) == 0 for pl in st.lists.values())
    u = F.fmm_apply(st, oracle_opset(1e-3, 1), f)
    assert rel_l2(u, direct_sum(pts, f)) < 1e-13


def test_planted_mistakes_break_the_pins(case4, monkeypatch):
    """Each plausible slip in the pass is caught by the direct-sum or symmetry pin."""
    pts, f, st, ref = case4
    ops = oracle_opset(1e-4, 1)
    # (1) a transposed D in L2T (incoming charges D instead of D^T)
    bad_lf = O.Skeleton(a=ops.lf.a, b=ops.lf.b, D=ops.lf.D.T.copy())
    bad = O.OpSet(tau=ops.tau, w_hi=ops.w_hi, hf=ops.hf, lf=bad_lf)
    assert rel_l2(F.fmm_apply(st, bad, f), ref) > 1e-2
    # (2) a sign error in the phase of the kernel used by the translations
    monkeypatch.setattr(F, "green", lambda x, y: np.conj(green(x, y)))
    assert rel_l2(F.fmm_apply(st, ops, f), ref) > 1e-2
    monkeypatch.undo()
    # (3) a dropped level of interaction lists
    st2 = build_structure(pts, 4.0)
    st2.lists[st2.tree.D].tgt = st2.lists[st2.tree.D].tgt[:0]
    st2.lists[st2.tree.D].src = st2.lists[st2.tree.D].src[:0]
    st2.lists[st2.tree.D].offset = st2.lists[st2.tree.D].offset[:0]
    assert rel_l2(F.fmm_apply(st2, ops, f), ref) > 1e-2


def test_cached_taus_lists_only_current_sets(tmp_path):
    """The baseline's lookup of cached oracle skeleton sets: a set counts only for
    its w_hi and the current oracle source hash."""
    import os

    from oracle.cache import _key, cached_taus

    for tau, w in [(1e-5, 4), (1e-3, 1), (2e-4, 4)]:
        open(_key(tau, w, str(tmp_path)), "wb").close()
    open(os.path.join(str(tmp_path), "oracle_opset_1.000e-06_4_0000000000.npz"), "wb").close()  # stale source
    assert sorted(cached_taus(4, str(tmp_path))) == [1e-5, 2e-4]
    assert cached_taus(1, str(tmp_path)) == [1e-3]
    assert cached_taus(2, str(tmp_path)) == []
