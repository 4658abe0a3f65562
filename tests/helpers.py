"""Shared test helpers: oracle operator sets (cached on disk) and injection into the library."""
from __future__ import annotations

from oracle import operators as O
from oracle.cache import oracle_opset  # noqa: F401  (re-exported for the tests)


def inject(ops: O.OpSet):
    """Copy an oracle operator set into a library OpSet (dfmm_opset_create / _set)."""
    from paper_1311_4257_amd import dfmm

    s = dfmm.OpSet.create(ops.tau, ops.w_hi)
    for w, sks in ops.hf.items():
        for d, sk in enumerate(sks):
            s.set(float(w), d, sk.a, sk.b, sk.D)
    s.set(0.5, 0, ops.lf.a, ops.lf.b, ops.lf.D)
    return s
