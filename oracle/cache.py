"""On-disk cache of oracle operator sets (test infrastructure only).

Values here are computed by ``oracle.operators`` and nothing else; they are
stored as plain .npz arrays (no pickle) keyed by (tau, w_hi) and a hash of the
operator module's source, so a change to the oracle invalidates them.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

from . import operators as O

DEFAULT_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", ".cache")


def _key(tau: float, w_hi: int, cache_dir: str) -> str:
    h = hashlib.sha1(open(O.__file__, "rb").read()).hexdigest()[:10]
    return os.path.join(cache_dir, f"oracle_opset_{tau:.3e}_{w_hi}_{h}.npz")


def cached_taus(w_hi: int, cache_dir: str = DEFAULT_DIR) -> list:
    """The tau values whose (tau, w_hi) operator set is cached for the current oracle source."""
    if not os.path.isdir(cache_dir):
        return []
    out = []
    for t in sorted(os.listdir(cache_dir)):
        parts = t[len("oracle_opset_"):-len(".npz")].split("_") if t.startswith("oracle_opset_") else []
        if len(parts) == 3 and parts[1] == str(w_hi) and os.path.join(cache_dir, t) == _key(float(parts[0]), w_hi,
                                                                                              cache_dir):
            out.append(float(parts[0]))
    return out


def oracle_opset(tau: float, w_hi: int, cache_dir: str = DEFAULT_DIR) -> O.OpSet:
    """The oracle's skeletons for (tau, w_hi), built once and cached."""
    fn = _key(tau, w_hi, cache_dir)
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
    try:  # the pivoted QRs of the build are large: let BLAS use every core
        from threadpoolctl import threadpool_limits

        with threadpool_limits(limits=os.cpu_count(), user_api="blas"):
            ops = O.build_opset(tau, w_hi)
    except ImportError:
        ops = O.build_opset(tau, w_hi)
    arrs = {"a_lf": ops.lf.a, "b_lf": ops.lf.b, "D_lf": ops.lf.D}
    for w, sks in ops.hf.items():
        for d, s in enumerate(sks):
            arrs[f"a_{w}_{d}"] = s.a
            arrs[f"b_{w}_{d}"] = s.b
            arrs[f"D_{w}_{d}"] = s.D
    os.makedirs(cache_dir, exist_ok=True)
    tmp = fn + ".tmp.npz"
    np.savez(tmp, **arrs)
    os.replace(tmp, fn)
    return ops
