"""Build the on-disk caches that the test suites read, ahead of a run (CPU only).

Two caches, both built on first use anyway and neither committed:
- tests/.cache: the oracle's skeleton sets and the oracle's float64 pass of
  the K = 16 injected-skeleton case (values from oracle/ only);
- .dfmm_cache: the library's own skeleton sets for the eps = 1e-4 and
  eps = 1e-6 float32 plans (tau = 1e-5 and 3e-8, up to w = 4), built by the
  library's host code through dfmm_opset_build, which needs no GPU.

The largest of them take minutes on a few cores.  Built inside a test, that
time passes in one fixture with nothing printed, so a cold GPU run looks
stalled; building them here first avoids that.

    python tests/build_caches.py
"""
from __future__ import annotations

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (tau, w_hi) of the oracle skeleton sets the CPU and GPU suites use
ORACLE_SETS = [(1e-3, 1), (1e-3, 2), (1e-3, 4), (1e-4, 1), (1e-4, 2), (1e-5, 4), (1e-6, 1)]
# (tau, w_hi) of the library's sets: the tau of eps = 1e-4 and eps = 1e-6 plans
LIBRARY_SETS = [(1e-5, 4), (3e-8, 4)]


def main() -> int:
    from tests.helpers import k16_case, oracle_opset

    t0 = time.perf_counter()
    for tau, w in ORACLE_SETS:
        oracle_opset(tau, w)
        print(f"oracle skeletons tau={tau:g} w={w}: {time.perf_counter() - t0:.0f} s", flush=True)
    k16_case()
    print(f"oracle pass of the K = 16 case: {time.perf_counter() - t0:.0f} s", flush=True)
    try:
        from paper_1311_4257_amd import dfmm
    except ImportError as e:  # the library is not built: its cache is left to the first plan
        print(f"library skeletons skipped: {e}", flush=True)
        return 0
    cache = os.path.join(ROOT, ".dfmm_cache")
    for tau, w in LIBRARY_SETS:
        dfmm.OpSet.build(tau, w, cache).close()
        print(f"library skeletons tau={tau:g} w={w}: {time.perf_counter() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
