"""GPU parity past the one-HF-level case: trees whose interaction lists reach
w = 2 (K = 8 sphere) or w = 4 (K = 16 sphere), so the w >= 2 transfers (HF-M2M
and HF-L2L through the wedge hierarchy of Figure 2), the w = 2 and 4 M2L, the
many-rhs leaf kernels (S2M in 32-rhs passes, L2T per leaf, the MFMA near
field) and the slot form of the translations all run.

With the oracle's skeletons injected (dfmm_opset_set) the library's pass is
compared element by element with the oracle's float64 pass of Algorithm 1; the
bound is float32 rounding of the translations (5e-6 relative L2 and max).
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle.fmm import fmm_apply
from oracle.kernel import direct_sum, rel_l2
from oracle.tree import build_structure
from paper_1311_4257_amd import workloads
from tests.helpers import inject, k16_case, oracle_opset

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".dfmm_cache")
BOUND = 5e-6


def _dfmm():
    from paper_1311_4257_amd import dfmm

    return dfmm


def _to_dev(f, cuda):
    import torch

    return torch.from_numpy(np.ascontiguousarray(f.astype(np.complex64))).to(cuda)


@pytest.fixture(scope="module")
def k8():
    pts = workloads.sphere_points(8192, 8.0, seed=8)
    st = build_structure(pts, 8.0)
    assert st.w_top == 2
    ops = oracle_opset(1e-4, 2)
    f = workloads.densities(len(pts), 32, seed=118)
    return pts, st, ops, f, fmm_apply(st, ops, f)


def _check(u, ref, what):
    u = u.astype(np.complex128)
    err = rel_l2(u, ref)
    worst = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
    print(f"{what}: rel L2 {err:.2e}  max {worst:.2e}")
    assert err < BOUND and worst < BOUND, (what, err, worst)


@pytest.mark.parametrize("nrhs,fused,prec", [(1, "0", 0), (1, "1", 0), (3, "0", 0), (1, "0", 1), (6, "1", 1),
                                             (16, "0", 0), (32, "0", 0)])
def test_injected_k8_matches_oracle(cuda, k8, monkeypatch, nrhs, fused, prec):
    """K = 8 sphere, oracle skeletons (tau = 1e-4, w = 1 and 2): pair form with and
    without the fused M2L (1-6 rhs, float32 and FP16X3 GEMMs) and slot form (16 and
    32 rhs) against the oracle's float64 pass."""
    pts, st, ops, f, ref = k8
    monkeypatch.setenv("DFMM_FUSED", fused)
    if nrhs >= 16:
        monkeypatch.setenv("DFMM_SLOT", "1")  # the slot form, also where the pair form costs less
    plan = _dfmm().Plan(pts, 8.0, opset=inject(ops), device=0, precision=prec)
    u = plan.apply(_to_dev(f[:nrhs], cuda)).cpu().numpy()
    _check(u, ref[:nrhs], f"K=8 injected nrhs={nrhs} fused={fused} prec={prec}")


@pytest.mark.parametrize("nrhs", [16, 32, 40])
def test_slot_form_equals_pair_form(cuda, monkeypatch, nrhs):
    """The slot form (every slot sums its terms in registers, float64 across
    terms) against the pair form (per-pair outputs, fixed-order float64
    reduction) on the library's own skeletons: the same sums in another
    rounding order; 40 rhs leaves a partial column tile.  Both are repeatable
    bit for bit and meet eps against the direct sum."""
    dfmm = _dfmm()
    pts = workloads.sphere_points(16384, 8.0, 41)
    f = workloads.densities(len(pts), nrhs, 52)
    fd = _to_dev(f, cuda)
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("DFMM_SLOT", mode)
        plan = dfmm.Plan(pts, 8.0, eps=1e-4, cache_dir=CACHE, device=0)
        a = plan.apply(fd).cpu().numpy()
        b = plan.apply(fd).cpu().numpy()
        assert np.array_equal(a, b)
        out[mode] = a.astype(np.complex128)
        plan.close()
    for k in range(nrhs):
        d = rel_l2(out["1"][k], out["0"][k])
        assert d < 1e-6, (k, d)
    tg = workloads.sample_targets(len(pts), 256, 53)
    ref = direct_sum(pts, f, tg)
    for mode in out:
        assert rel_l2(out[mode][:, tg], ref) <= 1e-4


def test_slot_form_column_chunks(cuda, monkeypatch):
    """16 rhs (one 16-column tile per slot) and 32 rhs (one 32-column tile) give the
    same columns to float32 rounding: a column's far-field arithmetic does not
    depend on the other columns of its tile."""
    monkeypatch.setenv("DFMM_SLOT", "1")
    pts = workloads.sphere_points(16384, 8.0, 61)
    f = workloads.densities(len(pts), 32, 62)
    plan = _dfmm().Plan(pts, 8.0, eps=1e-4, cache_dir=CACHE, device=0)
    u32 = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    u16 = plan.apply(_to_dev(f[8:24], cuda)).cpu().numpy()
    assert rel_l2(u16, u32[8:24]) < 1e-6, rel_l2(u16, u32[8:24])


@pytest.fixture(scope="module")
def k16():
    return k16_case()


@pytest.mark.parametrize("nrhs,fused,prec", [(1, "0", 0), (1, "1", 0), (1, "0", 1), (32, "0", 0)])
def test_injected_k16_matches_oracle(cuda, k16, monkeypatch, nrhs, fused, prec):
    """K = 16 sphere (HF levels w = 4, 2, 1: M2M 1 -> 2 -> 4 and L2L 4 -> 2 -> 1
    through the wedge hierarchy, M2L at w = 4, 2, 1), the oracle's tau = 1e-5
    skeletons (ranks up to 107): pair form at 1 rhs (separate and fused M2L,
    float32 and FP16X3 GEMMs) and slot form at 32 rhs, against the oracle."""
    pts, st, ops, f, ref = k16
    monkeypatch.setenv("DFMM_FUSED", fused)
    plan = _dfmm().Plan(pts, 16.0, opset=inject(ops), device=0, precision=prec)
    u = plan.apply(_to_dev(f[:nrhs], cuda)).cpu().numpy()
    _check(u, ref[:nrhs], f"K=16 injected nrhs={nrhs} fused={fused} prec={prec}")


@pytest.mark.parametrize("nrhs,form", [(16, "0"), (20, "0"), (31, "1"), (32, "1"), (40, "0")])
def test_default_form_follows_the_cost_rule(cuda, monkeypatch, nrhs, form):
    """Without DFMM_SLOT a float32 plan takes the slot form only where its work,
    padded to 32-column chunks, still costs less than the pair form's (30-32,
    59-64, ... rhs): the default apply equals the forced form bit for bit."""
    dfmm = _dfmm()
    pts = workloads.sphere_points(8192, 8.0, 71)
    fd = _to_dev(workloads.densities(len(pts), nrhs, 72), cuda)
    out = {}
    for mode in ("", form):
        monkeypatch.setenv("DFMM_SLOT", mode)
        plan = dfmm.Plan(pts, 8.0, eps=1e-4, cache_dir=CACHE, device=0)
        out[mode] = plan.apply(fd).cpu().numpy()
        plan.close()
    assert np.array_equal(out[""], out[form])
