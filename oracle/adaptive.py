"""Skeletons of the deeper low-frequency widths of an adaptive octree (Section 2.2).

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

The paper's octree is adaptive in the low-frequency regime: a box of width < 1
splits while it holds more than a fixed number of points, and the
low-frequency boxes use the kernel-independent FMM (one non-directional set
of equivalent and check points per box width; the Helmholtz kernel is not
scale invariant, so each width has its own).  The width-1/2 skeleton is built
with the directional ones (operators.build_opset); the widths 1/4, 1/8, ...
follow here by the same Eq. 2 construction:

  far region of width w: the boxes at the interaction-list offsets of width w
  (children of the parent's adjacent boxes, not adjacent themselves) plus the
  check points of the width-2w skeleton seen from each of the 8 child
  positions, so that LF-M2M and LF-L2L are accurate where the parent's
  skeleton is evaluated.
"""
from __future__ import annotations

import numpy as np

from .operators import OpSet, Skeleton, _sample_boxes, child_deltas, region_offsets, sample_sizes, skeleton


def deep_lf_skeletons(ops: OpSet, extra: int, seed: int = 12345) -> list:
    """Skeletons of the low-frequency widths 1/4, 1/8, ..., 2^-(1 + extra) at ops.tau."""
    deep = []
    parent, w = ops.lf, 0.25
    for k in range(extra):
        rng = np.random.default_rng([seed, 1, k])
        n_own, n_y = sample_sizes(w, ops.tau)
        dl = child_deltas(w)
        X = np.concatenate([_sample_boxes(rng, region_offsets(w) * w, w, n_own),
                            (parent.a[None, :, :] - dl[:, None, :]).reshape(-1, 3)], axis=0)
        Y = (rng.random((n_y, 3)) - 0.5) * w
        deep.append(skeleton(X, Y, ops.tau))
        parent, w = deep[-1], w / 2
    return deep


def lf_skeleton(ops: OpSet, deep: list, w: float) -> Skeleton:
    """The skeleton of a low-frequency box of width w <= 1/2."""
    k = int(round(np.log2(0.5 / w)))
    return ops.lf if k == 0 else deep[k - 1]
