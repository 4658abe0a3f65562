"""Shared test helpers: oracle operator sets (cached on disk) and injection into the library."""
from __future__ import annotations

from oracle import operators as O
from oracle.cache import oracle_opset  # noqa: F401  (re-exported for the tests)


def inject(ops: O.OpSet, deep=()):
    """Copy an oracle operator set into a library OpSet (dfmm_opset_create / _set);
    ``deep``: the oracle's skeletons of the LF widths 1/4, 1/8, ... (adaptive trees)."""
    from paper_1311_4257_amd import dfmm

    s = dfmm.OpSet.create(ops.tau, ops.w_hi)
    for w, sks in ops.hf.items():
        for d, sk in enumerate(sks):
            s.set(float(w), d, sk.a, sk.b, sk.D)
    s.set(0.5, 0, ops.lf.a, ops.lf.b, ops.lf.D)
    for k, sk in enumerate(deep):
        s.set(0.5 / 2 ** (k + 1), 0, sk.a, sk.b, sk.D)
    return s


def cached_oracle_pass(key: str, st, ops, f):
    """The oracle's pass of Algorithm 1 for (structure, skeletons, densities), computed
    by oracle.fmm only and kept as .npy under tests/.cache, keyed by the caller's
    key and a hash of the oracle's sources (a change to the oracle recomputes it)."""
    import hashlib
    import os

    import numpy as np

    from oracle import fmm as F
    from oracle.cache import DEFAULT_DIR

    h = hashlib.sha1()
    root = os.path.dirname(F.__file__)
    for name in ("fmm.py", "tree.py", "operators.py", "kernel.py"):
        with open(os.path.join(root, name), "rb") as fh:
            h.update(fh.read())
    fn = os.path.join(DEFAULT_DIR, f"oracle_pass_{key}_{h.hexdigest()[:10]}.npy")
    if os.path.exists(fn):
        return np.load(fn)
    u = F.fmm_apply(st, ops, f)
    os.makedirs(DEFAULT_DIR, exist_ok=True)
    tmp = fn + ".tmp.npy"
    np.save(tmp, u)
    os.replace(tmp, fn)
    return u


def k16_case():
    """The K = 16 injected-skeleton case: 16,384 points on the sphere of
    diameter 16 (seed 16, tree levels w = 4, 2, 1 and LF), the oracle's
    tau = 1e-5 skeletons up to w = 4, 32 rhs of densities (seed 116), and the
    oracle's float64 pass over them (cached)."""
    from oracle.tree import build_structure
    from paper_1311_4257_amd import workloads

    pts = workloads.sphere_points(16384, 16.0, seed=16)
    st = build_structure(pts, 16.0)
    assert st.w_top == 4
    ops = oracle_opset(1e-5, 4)
    f = workloads.densities(len(pts), 32, seed=116)
    return pts, st, ops, f, cached_oracle_pass("sphere16_16384_s16_f116_tau1e-5_w4", st, ops, f)
