"""The C ABI on the CPU: the library loads, exports every symbol declared in
include/dfmm.h, rejects bad input before touching a device, and builds its
float64 skeletons (host code) to the Eq. 2 accuracy."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dfmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dfmm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1311_4257_amd import dfmm

    lib = ctypes.CDLL(dfmm.LIB_PATH)
    names = _declared()
    assert "dfmm_plan" in names and "dfmm_apply" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dfmm.ABI_FUNCTIONS)


def test_header_constants_match_the_binding():
    from paper_1311_4257_amd import dfmm

    src = open(os.path.join(ROOT, "include", "dfmm.h")).read()
    m = re.search(r"#define DFMM_NOALLOC_MAX_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == dfmm.NOALLOC_MAX_BYTES
    m = re.search(r"#define DFMM_MAX_BATCH (\d+)", src)
    assert m and int(m.group(1)) == dfmm.MAX_BATCH


def test_bad_inputs_rejected_on_the_host():
    from paper_1311_4257_amd import dfmm

    good = np.zeros((4, 3))
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 3.0)                       # K not a power of two
    with pytest.raises(dfmm.DfmmError, match="EDOMAIN"):
        dfmm.Plan(np.array([[3.0, 0.0, 0.0]]), 4.0)   # |p| > K/2
    with pytest.raises(dfmm.DfmmError, match="EDOMAIN"):
        dfmm.Plan(np.array([[np.nan, 0.0, 0.0]]), 4.0)
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 4.0, eps=0.5)
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 4.0, eps=1e-7)             # below the float32 floor
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(np.zeros((0, 3)), 4.0)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.OpSet.build(1e-4, 3)                  # w_hi not a power of two
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, precision=7)           # unknown GEMM precision
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, eps=1e-6, precision=dfmm.PREC_FP16X3)  # split products need eps >= 1e-5
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 4.0, leaf_width=0.25)       # only the uniform leaf level of width 1/2
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, tol_factor=2.0)        # tau = tol_factor eps needs tol_factor in (0, 1]
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, tol_factor=-0.1)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, leaf_max=-1)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        dfmm.Plan(good, 4.0, leaf_max=16, lf_levels=7)  # at most 6 levels below width 1/2
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 4.0, leaf_max=16, precision=dfmm.PREC_FP16X3)  # adaptive trees: float32 only
    with pytest.raises(dfmm.DfmmError, match="EUNSUPPORTED"):
        dfmm.Plan(good, 4.0, eps=1e-6, leaf_max=16)  # ... and eps >= 1e-5 (the slot form)
    lib = dfmm._lib
    n = ctypes.c_size_t()
    assert lib.dfmm_workspace_bytes(None, 1, ctypes.byref(n)) == -1
    assert lib.dfmm_apply_ws(None, None, None, 1, None, 0, None) == -1
    assert lib.dfmm_apply_noalloc(None, None, None, 1, None) == -1
    arr = (ctypes.c_void_p * 1)(None)
    cnt = (ctypes.c_int * 1)(1)
    assert lib.dfmm_apply_batch(None, 1, arr, arr, cnt, None) == -1
    # the serving loop's entry points refuse null or empty arguments on the host
    srv = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 1)(None)
    assert lib.dfmm_server_create(None, 1, 1 << 30, 16, 0, ctypes.byref(srv)) == -1
    assert lib.dfmm_server_create(plans, 0, 1 << 30, 16, 0, ctypes.byref(srv)) == -1
    assert lib.dfmm_server_create(plans, 1, 1 << 30, 16, 0, ctypes.byref(srv)) == -1  # null plan
    assert lib.dfmm_server_create(plans, 1, 1 << 30, 0, 0, ctypes.byref(srv)) == -1   # max_batch_rhs
    assert lib.dfmm_server_create(plans, 1, 1 << 30, 16, 0, None) == -1
    t = ctypes.c_int64()
    assert lib.dfmm_server_submit(None, 0, None, None, 1, ctypes.byref(t)) == -1
    assert lib.dfmm_server_wait(None, 0, None, None) == -1
    assert lib.dfmm_server_drain(None) == -1
    assert lib.dfmm_server_passes(None, ctypes.byref(t)) == -1
    lib.dfmm_server_destroy(None)


def test_hbm_budget_refuses_a_plan_before_any_device_call():
    """hbm_budget_bytes: a plan that cannot fit is refused with DFMM_ENOMEM by a
    host-side check (this runs on a machine without a GPU, so a device call
    would fail with DFMM_EDEVICE instead); the message names both sizes."""
    from paper_1311_4257_amd import dfmm
    from paper_1311_4257_amd.workloads import sphere_points

    pts = sphere_points(1000, 4.0, seed=1)
    with pytest.raises(dfmm.DfmmError, match="ENOMEM") as ei:
        dfmm.Plan(pts, 4.0, hbm_budget_bytes=1000)
    assert "1000" in str(ei.value) and "hbm_budget_bytes" in str(ei.value)
    if not _gpu():   # within the budget the plan proceeds to the device
        with pytest.raises(dfmm.DfmmError, match="EDEVICE|ENOMEM"):
            dfmm.Plan(pts, 4.0, hbm_budget_bytes=1 << 40)


def _gpu() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_skeletons_meet_eq2_on_fresh_samples(tmp_path):
    from oracle import operators as O
    from paper_1311_4257_amd import dfmm

    tau = 1e-3
    s = dfmm.OpSet.build(tau, 1, str(tmp_path))
    s2 = dfmm.OpSet.build(tau, 1, str(tmp_path))   # second call reads the cache
    rng = np.random.default_rng(5)
    offs = O.region_offsets(1.0)
    dirs = np.array([O.direction(n, 1) for n in offs.tolist()])
    ranks = []
    for d in range(6):
        a, b, D = s.get(1.0, d)
        a2, b2, D2 = s2.get(1.0, d)
        assert np.array_equal(a, a2) and np.array_equal(D, D2)
        ranks.append(len(b))
        assert np.all(np.abs(b) <= 0.5 + 1e-12)        # equivalent points inside the box
        X = O._sample_boxes(rng, offs[dirs == d] * 1.0, 1.0, 600)
        Y = rng.random((300, 3)) - 0.5
        assert O.heldout_error(O.Skeleton(a=a, b=b, D=D), X, Y) < 10 * tau, d
    a, b, D = s.get(0.5, 0)
    X = O._sample_boxes(rng, O.region_offsets(0.5) * 0.5, 0.5, 600)
    Y = (rng.random((300, 3)) - 0.5) * 0.5
    assert O.heldout_error(O.Skeleton(a=a, b=b, D=D), X, Y) < 10 * tau
    # the oracle's ranks at the same tau are a cross-check (same criterion, own samples)
    from tests.helpers import oracle_opset

    orc = oracle_opset(tau, 1)
    assert abs(max(ranks) - orc.rank(1)) <= 0.15 * orc.rank(1)


def test_opset_roundtrip_and_injection(tmp_path):
    from paper_1311_4257_amd import dfmm

    s = dfmm.OpSet.create(1e-3, 1)
    rng = np.random.default_rng(1)
    for w, nd in [(1.0, 6), (0.5, 1)]:
        for d in range(nd):
            r = 5 + d
            s.set(w, d, rng.random((r, 3)), rng.random((r, 3)),
                  rng.random((r, r)) + 1j * rng.random((r, r)))
    p = str(tmp_path / "ops.bin")
    s.save(p)
    t = dfmm.OpSet.load(p)
    for w, nd in [(1.0, 6), (0.5, 1)]:
        for d in range(nd):
            for x, y in zip(s.get(w, d), t.get(w, d)):
                assert np.array_equal(x, y)
    assert t.info() == (1e-3, 1)
    # the deeper LF widths of adaptive trees (w = 1/4, 1/8, ...): set, read back;
    # a width not yet set is refused, and so are widths that are not LF widths
    for w in (0.25, 0.125):
        r = 4 if w == 0.25 else 3
        a, b = rng.random((r, 3)), rng.random((r, 3))
        Dm = rng.random((r, r)) + 1j * rng.random((r, r))
        s.set(w, 0, a, b, Dm)
        ga, gb, gD = s.get(w, 0)
        assert np.array_equal(ga, a) and np.array_equal(gb, b) and np.array_equal(gD, Dm)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        s.get(0.0625, 0)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        s.set(0.3, 0, a, b, Dm)
    with pytest.raises(dfmm.DfmmError, match="EINVAL"):
        s.set(0.25, 1, a, b, Dm)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of dfmm_options and dfmm_info have the C layout (gcc on the header)."""
    import shutil
    import subprocess

    from paper_1311_4257_amd import dfmm

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"dfmm_options": dfmm.Options, "dfmm_info": dfmm.Info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dfmm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)
