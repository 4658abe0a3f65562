"""GPU parity: libdfmm through its C ABI against the CPU float64 oracle.

* Structures (tree, lists, wedges, needed slots) must match the oracle bit for bit.
* With the oracle's own skeletons injected (dfmm_opset_set), the GPU matvec must
  reproduce the oracle's FMM element by element to float32 rounding.
* With the library's own skeletons, the matvec must meet eps against the
  float64 direct sum of Eq. 1.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle.fmm import fmm_apply
from oracle.kernel import direct_sum, rel_l2
from oracle.tree import build_structure
from paper_1311_4257_amd import workloads
from tests.helpers import inject, oracle_opset

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".dfmm_cache")


def _dfmm():
    from paper_1311_4257_amd import dfmm

    return dfmm


def _to_dev(f, cuda):
    import torch

    return torch.from_numpy(np.ascontiguousarray(f.astype(np.complex64))).to(cuda)


def _compare_structure(plan, st):
    dfmm = _dfmm()
    tr = st.tree
    assert np.array_equal(plan.export(dfmm.EXPORT_PERM), tr.perm)
    for l in range(tr.D + 1):
        lv = tr.levels[l]
        bx = plan.export(dfmm.EXPORT_BOXES, l)
        assert np.array_equal(bx[:, :3], lv.coords), l
        assert np.array_equal(bx[:, 3], lv.start) and np.array_equal(bx[:, 4], lv.end), l
    for l, pl in st.lists.items():
        pr = plan.export(dfmm.EXPORT_PAIRS, l)
        assert len(pr) == len(pl.tgt), l
        if len(pr):
            assert np.array_equal(pr[:, 0], pl.tgt) and np.array_equal(pr[:, 1], pl.src), l
            assert np.array_equal(pr[:, 2], pl.dir_in) and np.array_equal(pr[:, 3], pl.dir_out), l
    nr = plan.export(dfmm.EXPORT_NEAR)
    assert np.array_equal(nr[:, 0], st.near.tgt) and np.array_equal(nr[:, 1], st.near.src)
    for l in st.out_slots:
        assert np.array_equal(plan.export(dfmm.EXPORT_OUT_SLOTS, l), st.out_slots[l]), l
        assert np.array_equal(plan.export(dfmm.EXPORT_IN_SLOTS, l), st.in_slots[l]), l


def _structure_points(name, N):
    if name == "ellipsoid32":  # the serving mix's 4:2:1 ellipsoid in a K = 32 box
        return workloads.serving_points("ellipsoid", 32.0, N, 55), 32.0
    pts, _, cfg = workloads.make_config(name, N=N)
    return pts, cfg["K"]


@pytest.mark.parametrize("name,N", [("sphere4", 4096), ("sphere16", 16384), ("ellipsoid32", 131072)])
def test_structure_bit_exact(cuda, name, N):
    """Tree, lists, wedges and needed slots equal the oracle's bit for bit
    (the skeletons play no part here: the library builds its own)."""
    pts, K = _structure_points(name, N)
    st = build_structure(pts, K)
    plan = _dfmm().Plan(pts, K, eps=1e-4, cache_dir=CACHE, device=0)
    _compare_structure(plan, st)
    info = plan.info()
    assert info.w_top == st.w_top


def test_structure_points_on_dyadic_faces(cuda):
    """Points moved exactly onto box faces, edges and corners of every level
    (interior faces, the centre and the domain's boundary): the library's float64
    point -> box rule (interior faces to the upper box, the upper boundary
    clamped) must give the oracle's permutation, boxes, lists, wedges and
    slots bit for bit."""
    K = 8.0
    pts = workloads.sphere_points(8192, K, seed=71)
    rng = np.random.default_rng(72)
    st0 = build_structure(pts, K)
    D = st0.tree.D
    snapped = 0
    for i in rng.choice(len(pts), size=len(pts) // 2, replace=False):
        for ax in rng.choice(3, size=int(rng.integers(1, 4)), replace=False):
            lev = int(rng.integers(1, D + 1))
            h = K / 2 ** lev                           # faces of level lev: multiples of h
            pts[i, ax] = np.trunc(pts[i, ax] / h) * h  # towards 0, so |p| <= K/2 still holds
            snapped += 1
    pts[:4] = [[K / 2, 0, 0], [0, K / 2, 0], [0, 0, K / 2], [0, 0, 0]]   # upper boundary (clamped), centre
    pts[4:7] = [[-K / 2, 0, 0], [0, -K / 2, 0], [0, 0, -K / 2]]          # lower boundary
    edges = -K / 2 + (K / 2 ** D) * np.arange(2 ** D + 1)
    on_face = np.isin(pts, edges).any(axis=1)
    assert on_face.sum() >= len(pts) // 2 and snapped > len(pts) // 2
    st = build_structure(pts, K)
    plan = _dfmm().Plan(pts, K, eps=1e-4, cache_dir=CACHE, device=0)
    _compare_structure(plan, st)
    assert plan.info().w_top == st.w_top


@pytest.mark.parametrize("nrhs", [3, 32])
def test_dense_leaf_matches_oracle_fmm(cuda, nrhs):
    """One leaf of the K = 4 sphere holds 722 points (720 added uniformly in the
    middle fifth of a width-1/2 box): its targets span 12 blocks of the MFMA near
    field and of the MFMA L2T, and at 32 rhs its densities no longer fit the LDS
    block of the MFMA S2M, so S2M takes the VALU form.  With the oracle's
    skeletons on both sides the pass equals the oracle's float64 pass of the same
    tree to float32 rounding (3 rhs: pair form and VALU leaf kernels)."""
    pts, _, cfg = workloads.make_config("sphere4")
    K = cfg["K"]
    w = K / 2 ** build_structure(pts, K).tree.D
    c = (np.floor((0.8 * pts[0] + K / 2) / w) + 0.5) * w - K / 2
    rng = np.random.default_rng(907)
    pts = np.concatenate([pts, c + rng.uniform(-0.2 * w, 0.2 * w, size=(720, 3))])
    st = build_structure(pts, K)
    lv = st.tree.levels[st.tree.D]
    assert int(np.max(lv.end - lv.start)) == 722
    oops = oracle_opset(1e-4, 1)
    f = workloads.densities(len(pts), nrhs, 911)
    u_orc = fmm_apply(st, oops, f)
    plan = _dfmm().Plan(pts, K, opset=inject(oops), device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy().astype(np.complex128)
    err = rel_l2(u, u_orc)
    worst = np.max(np.abs(u - u_orc)) / np.max(np.abs(u_orc))
    print(f"dense leaf (722 points) nrhs={nrhs}: rel L2 {err:.2e}  max {worst:.2e}")
    assert err < 5e-6 and worst < 5e-6


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_flat_ellipsoid_meets_eps(cuda, eps):
    """The 4:2:1 ellipsoid of the serving mix (K = 32, N = 131,072, 129 points per
    square wavelength): the plan with the largest far-field share of the
    potential, closest to the eps bound."""
    pts = workloads.serving_points("ellipsoid", 32.0, 131072, 55)
    f = workloads.densities(len(pts), 2, 604)
    plan = _dfmm().Plan(pts, 32.0, eps=eps, cache_dir=CACHE, device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    tg = workloads.sample_targets(len(pts), 512, 704)
    err = rel_l2(u.astype(np.complex128)[:, tg], direct_sum(pts, f, tg))
    print(f"ellipsoid K=32 N=131072 eps={eps:g}: rel L2 {err:.2e}")
    assert err <= eps


@pytest.mark.parametrize("tau,prec,bound", [(1e-4, 0, 5e-6), (1e-6, 0, 5e-6), (1e-4, 1, 5e-6), (1e-4, 2, 2e-4)])
def test_injected_skeletons_match_oracle_fmm(cuda, tau, prec, bound):
    """Same skeletons on both sides: the GPU pass equals the oracle's float64 pass
    to float32 rounding (float32 and FP16X3 GEMMs), or to the 16 bits of BF16X3."""
    pts, f, cfg = workloads.make_config("sphere4")
    st = build_structure(pts, cfg["K"])
    oops = oracle_opset(tau, 1)
    u_orc = fmm_apply(st, oops, f)
    plan = _dfmm().Plan(pts, cfg["K"], opset=inject(oops), device=0, precision=prec)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy().astype(np.complex128)
    err = rel_l2(u, u_orc)
    worst = np.max(np.abs(u - u_orc)) / np.max(np.abs(u_orc))
    print(f"injected sphere4 tau={tau:g} precision {prec}: rel L2 {err:.2e}  max {worst:.2e}")
    assert err < bound
    assert worst < bound


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_sphere4_vs_direct_sum(cuda, eps):
    pts, f, cfg = workloads.make_config("sphere4")
    plan = _dfmm().Plan(pts, cfg["K"], eps=eps, cache_dir=CACHE, device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    err = rel_l2(u, direct_sum(pts, f))
    print(f"sphere4 eps={eps:g}: rel L2 vs direct sum {err:.2e}, ranks {list(plan.info().rank)[:4]}")
    assert err <= eps


def test_nrhs_batch_equals_single(cuda):
    """A column of a many-rhs apply equals the single-rhs apply of that column:
    bitwise while both take the VALU near field (3 rhs), to float32 rounding
    once the batch takes the MFMA near field (5 rhs: another summation order)."""
    pts, _, cfg = workloads.make_config("sphere4", N=2048)
    f = workloads.densities(len(pts), 5, seed=7)
    plan = _dfmm().Plan(pts, cfg["K"], opset=inject(oracle_opset(1e-3, 1)), device=0)
    u1 = [plan.apply(_to_dev(f[j:j + 1], cuda)).cpu().numpy()[0] for j in range(5)]
    u3 = plan.apply(_to_dev(f[:3], cuda)).cpu().numpy()
    for j in range(3):
        assert np.array_equal(u1[j], u3[j]), j
    u5 = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    for j in range(5):
        d = np.linalg.norm(u5[j] - u1[j]) / np.linalg.norm(u1[j])
        assert d <= 1e-6, (j, d)


@pytest.mark.parametrize("eps,nrhs", [(1e-4, 1), (1e-4, 5), (1e-4, 20), (1e-4, 40), (1e-6, 1), (1e-6, 3)])
def test_near_field_only_close_pairs(cuda, eps, nrhs):
    """Points in two adjacent leaves only (so every pair is near field), with
    pairs 1e-3 .. 1e-2 apart: the pass is the direct sum up to float32 rounding.
    One leaf holds 160 points (two target blocks of the MFMA near field, which
    fast plans take from 4 right-hand sides on; 20 and 40 rhs are one and two
    column groups of 32)."""
    rng = np.random.default_rng(11)
    a = rng.uniform(0.02, 0.48, (120, 3)) + np.array([0.0, 0.0, 0.0])
    b = rng.uniform(0.02, 0.48, (120, 3)) + np.array([0.5, 0.0, 0.0])
    close = a[:40] + rng.normal(0, 1, (40, 3)) * 3e-3       # close partners of the first 40 of a
    pts = np.concatenate([a, b, np.clip(close, 0.001, 0.499)])
    f = (rng.standard_normal((nrhs, len(pts))) + 1j * rng.standard_normal((nrhs, len(pts)))).astype(np.complex128)
    plan = _dfmm().Plan(pts, 4.0, eps=eps, cache_dir=CACHE, device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    ref = direct_sum(pts, f, np.arange(len(pts)))
    err = rel_l2(u, ref)
    worst = max(rel_l2(u[k:k + 1], ref[k:k + 1]) for k in range(nrhs))
    print(f"near field only, eps={eps:g}, nrhs={nrhs}: rel L2 {err:.2e}, worst rhs {worst:.2e}")
    assert err < 1e-6 and worst < 1e-6


def test_back_to_back_applies_on_a_stream(cuda):
    """Applies enqueued back to back (no host wait) on a non-default stream give
    bitwise the results of separately synchronized applies: the near-field
    stream forks from and joins into the caller's stream."""
    import torch

    pts, f, cfg = workloads.make_config("sphere4")
    plan = _dfmm().Plan(pts, cfg["K"], eps=1e-4, cache_dir=CACHE, device=0)
    rng = np.random.default_rng(5)
    fs = [_to_dev((rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape)), cuda) for _ in range(4)]
    ref = []
    for x in fs:
        ref.append(plan.apply(x).cpu().numpy())
        torch.cuda.synchronize()
    stream = torch.cuda.Stream(device=cuda)
    us = [torch.empty_like(x) for x in fs]
    with torch.cuda.stream(stream):
        for _ in range(3):
            for x, u in zip(fs, us):
                plan.apply(x, u, stream)
    stream.synchronize()
    for u, r in zip(us, ref):
        assert np.array_equal(u.cpu().numpy(), r)


def test_graph_captured_apply_replays_match_eager(cuda):
    """An apply captured into a HIP graph (after one uncaptured apply with the same
    nrhs) replays bitwise equal to eager applies, with eager work and host
    synchronisation between the replays, also after a larger apply has grown
    the plan's workspace; capturing first is refused."""
    import torch

    pts, _, cfg = workloads.make_config("sphere4")
    N = pts.shape[0]
    plan = _dfmm().Plan(pts, cfg["K"], eps=1e-4, cache_dir=CACHE, device=0)
    rng = np.random.default_rng(7)

    def dens():
        return _to_dev(rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N)), cuda)

    x = dens()
    u = torch.empty_like(x)
    g0 = torch.cuda.CUDAGraph()
    with pytest.raises(_dfmm().DfmmError):
        with torch.cuda.graph(g0):
            u.zero_()
            plan.apply(x, u)
    xs = [dens() for _ in range(3)]
    eager = []
    for xx in xs:
        eager.append(plan.apply(xx).cpu().numpy())
        torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.apply(x, u)
    for _ in range(2):
        for xx, ref in zip(xs, eager):
            x.copy_(xx)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(u.cpu().numpy(), ref)
    # the eager path still works after the capture
    assert np.array_equal(plan.apply(xs[0]).cpu().numpy(), eager[0])
    # a larger apply grows the workspace; the graph still addresses the old one,
    # which the plan keeps, so replays stay equal to the eager results
    big = _to_dev(rng.standard_normal((12, N)) + 1j * rng.standard_normal((12, N)), cuda)
    plan.apply(big)
    torch.cuda.synchronize()
    for xx, ref in zip(xs, eager):
        x.copy_(xx)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref)


def test_repeat_is_bitwise_deterministic(cuda):
    pts, f, cfg = workloads.make_config("sphere4", N=2048)
    plan = _dfmm().Plan(pts, cfg["K"], opset=inject(oracle_opset(1e-3, 1)), device=0)
    fd = _to_dev(f, cuda)
    a = plan.apply(fd).cpu().numpy()
    b = plan.apply(fd).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nrhs,prec,tau", [(1, 0, 1e-3), (5, 0, 1e-3), (1, 1, 1e-3), (5, 2, 1e-3), (3, 0, 1e-6)])
def test_gemm_launch_shapes_do_not_change_results(cuda, tmp_path, nrhs, prec, tau):
    """Every GEMM launch shape (16-64 columns per workgroup, M-slices, 4- or
    2-wave workgroups, operator staged in LDS or not, fused M2L) gives the same
    potentials bit for bit, in float32 and in the split 16-bit GEMMs: a shape
    only regroups whole columns and whole 16-row tiles, every output entry
    keeps its order of products, and the 16-bit scales are per operator and
    per column.  The shapes are forced through the tuning record that the
    first apply wrote."""
    import glob

    dfmm = _dfmm()
    pts, _, cfg = workloads.make_config("sphere4", N=2048)
    f = workloads.densities(len(pts), nrhs, 707)
    ops = inject(oracle_opset(tau, 1))  # tau = 1e-6: a precise plan (float64 partial sums)
    fd = _to_dev(f, cuda)
    plan = dfmm.Plan(pts, cfg["K"], opset=ops, cache_dir=str(tmp_path), device=0, precision=prec)
    ref = plan.apply(fd).cpu().numpy()
    recs = glob.glob(str(tmp_path / "dfmm_tune_*.txt"))
    assert len(recs) == 1
    n = int(open(recs[0]).read().split()[2])
    shapes = [(1, 1, 0, 4, 0), (2, 2, 0, 4, 0), (3, 1, 0, 4, 0), (4, 3, 0, 4, 0), (3, 2, 1, 4, 0),
              (1, 4, 0, 2, 0), (4, 1, 0, 2, 0), (2, 1, 0, 4, 4), (3, 1, 0, 4, 1)]
    if tau < 3e-6:  # precise plans: no operator staging in LDS, no fused M2L
        shapes = [sh for sh in shapes if sh[2] == 0 and sh[4] == 0]
    for nt, sl, alds, nw, fused in shapes:
        text = f"dfmm-tune 4 {n}\n" + f"{nt} {sl} {alds} {nw}\n" * n + f"fused {fused}\n"
        with open(recs[0], "w") as fh:
            fh.write(text)
        p2 = dfmm.Plan(pts, cfg["K"], opset=ops, cache_dir=str(tmp_path), device=0, precision=prec)
        u = p2.apply(fd).cpu().numpy()
        assert open(recs[0]).read() == text, "the forced shape was not taken"
        assert np.array_equal(u, ref), (nt, sl, alds, nw, fused)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_sphere16_full_size_sampled_targets(cuda, eps):
    """The benchmark workload (K = 16 sphere, N = 65,536) with the eps = 1e-4 and the
    eps = 1e-6 plan, on 2,048 sampled targets against the direct sum."""
    pts, f, cfg = workloads.make_config("sphere16")
    plan = _dfmm().Plan(pts, cfg["K"], eps=eps, cache_dir=CACHE, device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    tg = workloads.sample_targets(len(pts), cfg["n_check"], cfg["check_seed"])
    err = rel_l2(u[:, tg], direct_sum(pts, f, tg))
    print(f"sphere16 eps={eps:g}: rel L2 vs direct sum on {len(tg)} targets {err:.2e}, "
          f"ranks {[plan.info().rank[l] for l in range(plan.info().depth + 1)]}")
    assert err <= eps


def test_ellipsoid32_nrhs32_sampled_targets(cuda):
    """4:2:1 ellipsoid, K = 32, N = 262,144 area-uniform points, 32 right-hand sides in
    one apply, eps = 1e-4; 2,048 sampled targets (seed 303) x 32 rhs against the
    direct sum: the benchmark's workload in its launch configuration."""
    pts, f, cfg = workloads.make_config("ellipsoid32")
    plan = _dfmm().Plan(pts, cfg["K"], eps=cfg["eps"], cache_dir=CACHE, device=0)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    tg = workloads.sample_targets(len(pts), cfg["n_check"], cfg["check_seed"])
    ref = direct_sum(pts, f, tg)
    err = rel_l2(u[:, tg], ref)
    worst = max(rel_l2(u[k, tg], ref[k]) for k in range(f.shape[0]))
    print(f"ellipsoid32 nrhs=32: rel L2 {err:.2e} (worst rhs {worst:.2e}), w_top {plan.info().w_top}")
    assert err <= cfg["eps"]


@pytest.mark.parametrize("nrhs", [1, 6])
def test_split_precision_plans(cuda, nrhs):
    """FP16X3 / BF16X3 translation GEMMs (hi/lo 16-bit products, float32 sums)
    against the float32 plan on the same skeletons: FP16X3 (scaled, 22-bit
    operands) to float32 level, BF16X3 (16-bit operands) to ~1e-5; both within
    eps of the direct sum.  Split precision is refused for precise plans."""
    dfmm = _dfmm()
    pts = workloads.sphere_points(16384, 8.0, 31)
    f = workloads.densities(len(pts), nrhs, 32)
    fd = _to_dev(f, cuda)
    tg = workloads.sample_targets(len(pts), 512, 33)
    ref = direct_sum(pts, f, tg)
    u = {}
    for prec in (dfmm.PREC_FP32, dfmm.PREC_FP16X3, dfmm.PREC_BF16X3):
        plan = dfmm.Plan(pts, 8.0, eps=1e-4, cache_dir=CACHE, device=0, precision=prec)
        u[prec] = plan.apply(fd).cpu().numpy().astype(np.complex128)
    d16 = rel_l2(u[dfmm.PREC_FP16X3], u[dfmm.PREC_FP32])
    dbf = rel_l2(u[dfmm.PREC_BF16X3], u[dfmm.PREC_FP32])
    errs = {p: rel_l2(v[:, tg], ref) for p, v in u.items()}
    print(f"nrhs={nrhs}: fp16x3 vs fp32 {d16:.2e}, bf16x3 vs fp32 {dbf:.2e}, vs direct sum {errs}")
    assert d16 < 2e-6
    assert dbf < 1e-4
    assert all(e <= 1e-4 for e in errs.values())
    with pytest.raises(dfmm.DfmmError):
        dfmm.Plan(pts[:512] / 2, 4.0, eps=1e-6, cache_dir=CACHE, device=0, precision=dfmm.PREC_FP16X3)


@pytest.mark.parametrize("prec,nrhs,bound", [(1, 8, 1e-6), (1, 40, 1e-6), (2, 8, 1e-4)])
def test_near_field_split_precision(cuda, prec, nrhs, bound):
    """The MFMA near field with split 16-bit products (tile-scaled G, column-scaled
    densities) on the two-leaf geometry with pairs 1e-3 .. 1e-2 apart: FP16X3 to
    float32 level, BF16X3 to its 16 bits, against the direct sum."""
    rng = np.random.default_rng(11)
    a = rng.uniform(0.02, 0.48, (120, 3))
    b = rng.uniform(0.02, 0.48, (120, 3)) + np.array([0.5, 0.0, 0.0])
    close = a[:40] + rng.normal(0, 1, (40, 3)) * 3e-3
    pts = np.concatenate([a, b, np.clip(close, 0.001, 0.499)])
    f = (rng.standard_normal((nrhs, len(pts))) + 1j * rng.standard_normal((nrhs, len(pts)))).astype(np.complex128)
    plan = _dfmm().Plan(pts, 4.0, eps=1e-4, cache_dir=CACHE, device=0, precision=prec)
    u = plan.apply(_to_dev(f, cuda)).cpu().numpy()
    err = rel_l2(u, direct_sum(pts, f, np.arange(len(pts))))
    print(f"near field only, precision {prec}, nrhs={nrhs}: rel L2 {err:.2e}")
    assert err < bound


def test_degenerate_inputs(cuda):
    """Edge cases of the boundary: one point (u = 0 exactly), coincident points
    (G := 0 at r = 0), points exactly on |p| = K/2 including the positive axis
    tips (clamped into the last box), and domains too small for any HF level
    (K = 1 and 2: only the LF level, or only the near field), against the
    direct sum."""
    dfmm = _dfmm()
    rng = np.random.default_rng(21)

    def run(pts, K, nrhs=2):
        f = (rng.standard_normal((nrhs, len(pts))) + 1j * rng.standard_normal((nrhs, len(pts))))
        plan = dfmm.Plan(pts, K, eps=1e-4, cache_dir=CACHE, device=0)
        u = plan.apply(_to_dev(f, cuda)).cpu().numpy().astype(np.complex128)
        return u, direct_sum(pts, f.astype(np.complex64).astype(np.complex128), np.arange(len(pts))), plan

    u, ref, _ = run(np.array([[0.3, -0.2, 0.1]]), 2.0)
    assert np.all(u == 0)
    u, ref, _ = run(np.array([[0.25, 0.25, 0.25]] * 3), 2.0)  # three coincident points
    assert np.all(u == 0)
    pts = np.concatenate([np.array([[0.1, 0.1, 0.1]] * 2), rng.uniform(-0.5, 0.5, (30, 3))])
    u, ref, _ = run(pts, 2.0)
    assert rel_l2(u, ref) < 1e-6
    K = 8.0
    axis = np.array([[K / 2, 0, 0], [-K / 2, 0, 0], [0, K / 2, 0], [0, -K / 2, 0], [0, 0, K / 2], [0, 0, -K / 2]])
    pts = np.concatenate([axis, workloads.sphere_points(3000, K, 22)])
    u, ref, plan = run(pts, K)
    err = rel_l2(u, ref)
    print(f"boundary points K=8: rel L2 {err:.2e}, w_top {plan.info().w_top}")
    assert err <= 1e-4
    for K, n in ((1.0, 40), (2.0, 600)):
        pts = workloads.sphere_points(n, K, 23)
        u, ref, plan = run(pts, K, nrhs=5)
        err = rel_l2(u, ref)
        print(f"K={K:g} N={n}: rel L2 {err:.2e}, w_top {plan.info().w_top}, depth {plan.info().depth}")
        assert err <= 1e-4


@pytest.mark.parametrize("prec,nrhs", [(0, 1), (0, 5), (1, 3)])
def test_fused_m2l_equals_separate_launches(cuda, prec, nrhs, monkeypatch):
    """Every level's M2L in one launch (own pair scratch per level, reductions in
    the same order) gives bitwise the result of the separate launches."""
    dfmm = _dfmm()
    pts = workloads.sphere_points(16384, 8.0, 41)
    f = workloads.densities(len(pts), nrhs, 42)
    fd = _to_dev(f, cuda)
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("DFMM_FUSED", mode)
        plan = dfmm.Plan(pts, 8.0, eps=1e-4, cache_dir=CACHE, device=0, precision=prec)
        out[mode] = plan.apply(fd).cpu().numpy()
        plan.close()
    assert np.array_equal(out["0"], out["1"])
    tg = workloads.sample_targets(len(pts), 256, 43)
    assert rel_l2(out["1"].astype(np.complex128)[:, tg], direct_sum(pts, f, tg)) <= 1e-4
