"""Shared test helpers: oracle operator sets (cached on disk) and injection into the library.

The cache holds only values computed by ``oracle/`` (never by the library).
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

from oracle import operators as O

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), ".cache")


def _key(tau: float, w_hi: int) -> str:
    src = open(O.__file__, "rb").read()
    h = hashlib.sha1(src).hexdigest()[:10]
    return os.path.join(CACHE, f"oracle_opset_{tau:.3e}_{w_hi}_{h}.npz")


def oracle_opset(tau: float, w_hi: int) -> O.OpSet:
    """The oracle's skeletons for (tau, w_hi), cached as .npz (plain arrays, no pickle)."""
    fn = _key(tau, w_hi)
    if os.path.exists(fn):
        z = np.load(fn)
        hf = {}
        w = 1
        while w <= w_hi:
            hf[w] = [O.Skeleton(a=z[f"a_{w}_{d}"], b=z[f"b_{w}_{d}"], D=z[f"D_{w}_{d}"])
                     for d in range(6 * w * w)]
            w *= 2
        lf = O.Skeleton(a=z["a_lf"], b=z["b_lf"], D=z["D_lf"])
        return O.OpSet(tau=tau, w_hi=w_hi, hf=hf, lf=lf)
    ops = O.build_opset(tau, w_hi)
    arrs = {"a_lf": ops.lf.a, "b_lf": ops.lf.b, "D_lf": ops.lf.D}
    for w, sks in ops.hf.items():
        for d, s in enumerate(sks):
            arrs[f"a_{w}_{d}"] = s.a
            arrs[f"b_{w}_{d}"] = s.b
            arrs[f"D_{w}_{d}"] = s.D
    os.makedirs(CACHE, exist_ok=True)
    tmp = fn + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, fn)
    return ops


def inject(ops: O.OpSet):
    """Copy an oracle operator set into a library OpSet (dfmm_opset_create / _set)."""
    from paper_1311_4257_amd import dfmm

    s = dfmm.OpSet.create(ops.tau, ops.w_hi)
    for w, sks in ops.hf.items():
        for d, sk in enumerate(sks):
            s.set(float(w), d, sk.a, sk.b, sk.D)
    s.set(0.5, 0, ops.lf.a, ops.lf.b, ops.lf.D)
    return s
