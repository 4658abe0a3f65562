"""GPU: the adaptive low-frequency tree (Section 2.2; dfmm_options.leaf_max).

A box of width <= 1/2 splits while it holds more than leaf_max points, down to
three levels below width 1/2; LF-M2M runs up the LF levels, LF-M2L and LF-L2L
down them (Algorithm 1's LF loops), each width with its own skeleton, and
leaves of different sizes that are adjacent at the coarser one's level are
summed directly in the near field.

* Structure against the oracle (oracle.tree.build_structure with the same
  leaf_max): the permutation, the boxes of every level, the M2L pairs of the
  levels below width 1/2, the leaves and the near-field pairs, bit for bit.
* With the oracle's skeletons injected (every LF width included) the pass must
  equal the oracle's float64 pass over the same adaptive tree to float32
  rounding: 5e-6 relative L2 and max, at 1, 3, 20 and 32 rhs (32: the
  MFMA S2M, whose leaves sit at several LF levels).
* With the library's own skeletons the pass must meet eps against the float64
  direct sum of Eq. 1.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import fmm as F
from oracle import tree as T
from oracle.adaptive import deep_lf_skeletons
from oracle.kernel import direct_sum, rel_l2
from paper_1311_4257_amd import workloads
from tests.helpers import inject, oracle_opset

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".dfmm_cache")
LEAF_MAX = 16
TAU = 1e-4


def _dfmm():
    from paper_1311_4257_amd import dfmm

    return dfmm


def _dev(f, cuda):
    import torch

    return torch.from_numpy(np.ascontiguousarray(f.astype(np.complex64))).to(cuda)


@pytest.fixture(scope="module")
def case():
    """A dense K = 4 sphere (N = 12,000): width-1/2 boxes hold ~45 points, so the
    tree reaches widths 1/8 and 1/16."""
    pts = workloads.sphere_points(12000, 4.0, seed=41)
    st = T.build_structure(pts, 4.0, leaf_max=LEAF_MAX, extra=3)
    ops = oracle_opset(TAU, 1)
    deep = deep_lf_skeletons(ops, st.tree.Dmax - st.tree.D)
    return pts, st, ops, deep


def test_adaptive_structure_matches_oracle(cuda, case):
    dfmm = _dfmm()
    pts, st, ops, deep = case
    tr = st.tree
    plan = dfmm.Plan(pts, 4.0, opset=inject(ops, deep), device=0, leaf_max=LEAF_MAX)
    info = plan.info()
    assert info.depth == tr.D and info.depth_max == tr.Dmax
    assert np.array_equal(plan.export(dfmm.EXPORT_PERM), tr.perm)
    for l in range(tr.Dmax + 1):
        lv = tr.levels[l]
        bx = plan.export(dfmm.EXPORT_BOXES, l)
        assert np.array_equal(bx[:, :3], lv.coords), l
        assert np.array_equal(bx[:, 3], lv.start) and np.array_equal(bx[:, 4], lv.end), l
    for l in range(tr.D + 1, tr.Dmax + 1):
        pr = plan.export(dfmm.EXPORT_PAIRS, l)
        pl = st.lists[l]
        assert len(pr) == len(pl.tgt) > 0, l
        assert np.array_equal(pr[:, 0], pl.tgt) and np.array_equal(pr[:, 1], pl.src), l
    lv_exp = plan.export(dfmm.EXPORT_LEAVES)
    leaves = [(int(l), int(b)) for l, b in lv_exp[:, :2]]
    assert sorted(leaves) == sorted(tr.leaf_boxes())
    assert np.array_equal(lv_exp[:, 2], np.sort(lv_exp[:, 2]))  # point order
    for (l, b), s, e in zip(leaves, lv_exp[:, 2], lv_exp[:, 3]):
        assert tr.levels[l].start[b] == s and tr.levels[l].end[b] == e
    near = plan.export(dfmm.EXPORT_NEAR)
    got = sorted((leaves[B], leaves[A]) for B, A in near.tolist())
    assert got == sorted(st.near)
    assert any(B[0] != A[0] for B, A in got)        # coarse-fine pairs are there
    assert info.leaves == len(leaves)


@pytest.mark.parametrize("nrhs", [1, 3, 20, 32])
def test_adaptive_injected_matches_oracle_pass(cuda, case, nrhs):
    """The oracle's skeletons of every width on both sides: the GPU pass against
    the oracle's float64 pass of the same adaptive tree, element by element."""
    dfmm = _dfmm()
    pts, st, ops, deep = case
    f = workloads.densities(len(pts), nrhs, seed=140 + nrhs)
    ref = F.fmm_apply(st, ops, f, deep=deep)
    plan = dfmm.Plan(pts, 4.0, opset=inject(ops, deep), device=0, leaf_max=LEAF_MAX)
    u = plan.apply(_dev(f, cuda)).cpu().numpy()
    err = rel_l2(u, ref)
    worst = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print(f"adaptive injected nrhs={nrhs}: rel L2 {err:.2e}  max {worst:.2e}")
    assert err < 5e-6 and worst < 5e-6


def test_adaptive_plan_meets_eps(cuda, case):
    """The library's own skeletons (widths 1/2 .. 1/16 built by its precompute):
    every target against the float64 direct sum at eps = 1e-4, 2 rhs."""
    dfmm = _dfmm()
    pts = case[0]
    f = workloads.densities(len(pts), 2, seed=150)
    plan = dfmm.Plan(pts, 4.0, eps=1e-4, cache_dir=CACHE, device=0, leaf_max=LEAF_MAX)
    u = plan.apply(_dev(f, cuda)).cpu().numpy()
    err = rel_l2(u, direct_sum(pts, f))
    print(f"adaptive own skeletons: rel L2 {err:.2e}, leaves {plan.info().leaves}")
    assert err <= 1e-4


def test_adaptive_without_splits_equals_uniform(cuda):
    """leaf_max above every box count: no box splits, the leaves are the boxes of
    width 1/2, and the result equals the uniform plan's to float32 rounding
    (only the order of points inside a leaf, sorted by a finer key, differs)."""
    dfmm = _dfmm()
    pts, _, cfg = workloads.make_config("sphere4")
    f = workloads.densities(len(pts), 2, seed=151)
    ops = inject(oracle_opset(TAU, 1))
    u0 = dfmm.Plan(pts, 4.0, opset=ops, device=0).apply(_dev(f, cuda)).cpu().numpy()
    pa = dfmm.Plan(pts, 4.0, opset=ops, device=0, leaf_max=10 ** 6)
    assert pa.info().depth_max == pa.info().depth
    u1 = pa.apply(_dev(f, cuda)).cpu().numpy()
    assert rel_l2(u1, u0) < 1e-6
