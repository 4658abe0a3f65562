"""Directional skeletons (a, b, D) of Eq. (2) by pivoted QR (Section 2.1).

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

For a box Y of width w centred at 0 and a far region X, Eq. (2) asks for
equivalent points b in Y, check points a in X and a matrix D with
G(x, y) ~= sum_q G(x, b_q) sum_p D_qp G(a_p, y) for x in X, y in Y.  The
paper refers to a random sampling method based on pivoted QR; the reading
used here (same steps in the same order as that description):

  1. sample Y (uniform in the box) and X (the far region, below);
  2. column-pivoted QR of G(X, Y), truncated at the first rank r whose
     residual has Frobenius norm <= tau ||G(X, Y)||_F; b = the first r pivot
     columns;
  3. column-pivoted QR of G(X, Y)^T; a = the first r pivot rows;
  4. D = G(X, b)^+ G(X, Y) G(a, Y)^+ (float64 SVD pseudo-inverses).

Outgoing use (Section 2.1): check potentials at a, equivalent charges
D (check potentials), equivalent points b.  Incoming use: check points b,
equivalent points a, charges D^T (check potentials).

Far regions (Section 2.2: wedges of angle O(1/w) overlapping hierarchically,
Figure 2; readings):

* HF width w, direction l: the boxes at offsets n (units of w) that can be in
  an interaction list at width w (S(n) > T(w) and, for some child position o,
  the parent offset floor((o + n)/2) has S <= T(2w)) and whose wedge is l;
  plus the check points a of every direction l' at width 2w with
  l'↓ = l, translated by -delta_o for each of the 8 child positions o
  (delta_o = (o - 1/2) w), so that HF-M2M and HF-L2L are accurate exactly
  where the parent's skeleton is evaluated.  Widths are built top-down from
  w_hi, the largest width of the set.
* LF (w = 1/2): the V-list boxes (adjacency at the leaf and parent levels)
  plus the check points of all 6 directions at width 1, translated likewise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .kernel import green
from .tree import direction, direction_down, near_limit4, near_sum

# sample sizes (oracle's own choice; any adequate sampling gives a valid skeleton).
# Wider boxes have more wavelengths across them and wider far regions, and
# tighter tolerances resolve finer detail, so both samples grow with w and 1/tau.
N_Y = 900            # candidate equivalent points in a box of width <= 1
N_OWN = 1200         # points drawn in the region's own boxes, per unit width
MIN_PER_BOX = 6


def sample_sizes(w: float, tau: float):
    """(points in the far region's own boxes, candidate points in the box)."""
    ww = max(1.0, float(w))
    n_own = N_OWN * ww
    n_y = N_Y * (1.0 + 0.35 * np.log2(ww))
    if tau < 1e-6:
        n_own *= 2.5
        n_y *= 16.0 / 9.0
    return int(round(n_own)), int(round(n_y))


@dataclass
class Skeleton:
    a: np.ndarray       # (r, 3) check points, box frame
    b: np.ndarray       # (r, 3) equivalent points, box frame
    D: np.ndarray       # (r, r) complex128
    X: np.ndarray = field(default=None, repr=False)   # the far samples used

    @property
    def r(self) -> int:
        return self.b.shape[0]


@dataclass
class OpSet:
    tau: float
    w_hi: int
    hf: dict            # w -> list of Skeleton, one per direction (6 w^2)
    lf: Skeleton

    def rank(self, w) -> int:
        if w < 1:
            return self.lf.r
        return max(s.r for s in self.hf[int(w)])


def region_offsets(w: float) -> np.ndarray:
    """Offsets n that can occur in an interaction list at width w."""
    lim = near_limit4(w)
    lim2 = near_limit4(2 * w)
    rp = 0
    while 4 * (2 * (rp + 1) - 1) ** 2 <= lim2:
        rp += 1
    r = 2 * rp + 2
    g = np.arange(-r, r + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    n = n[4 * near_sum(n) > lim]
    ok = np.zeros(len(n), dtype=bool)
    for o in range(8):
        ov = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1])
        m = np.floor_divide(n + ov, 2)
        ok |= 4 * near_sum(m) <= lim2
    return n[ok]


def child_deltas(w: float) -> np.ndarray:
    """delta_o = (o - 1/2) w: centre of the child at octant o relative to its parent."""
    o = np.arange(8)
    ov = np.stack([o & 1, (o >> 1) & 1, (o >> 2) & 1], axis=1).astype(np.float64)
    return (ov - 0.5) * w


def _sample_boxes(rng, centres: np.ndarray, w: float, n_total: int) -> np.ndarray:
    k = max(MIN_PER_BOX, -(-n_total // max(1, len(centres))))
    u = rng.random((len(centres), k, 3)) - 0.5
    return (centres[:, None, :] + w * u).reshape(-1, 3)


def skeleton(X: np.ndarray, Y: np.ndarray, tau: float) -> Skeleton:
    """Steps 2-4 above for the sample sets X (far) and Y (box).

    The rank is the smallest r whose trailing block of R has Frobenius norm
    <= tau ||R||_F (the residual of projecting G(X, Y) on the r pivot columns);
    D = G(X, b)^+ G(X, Y) G(a, Y)^+ is the middle factor that best reproduces
    G(X, Y) from the chosen columns and rows.
    """
    M = green(X, Y)
    R, piv = sla.qr(M, mode="r", pivoting=True)
    rows = np.sum(np.abs(np.triu(R)) ** 2, axis=1)
    tail = np.sqrt(np.cumsum(rows[::-1])[::-1])      # tail[k] = ||R[k:, k:]||_F
    ok = np.nonzero(tail <= tau * tail[0])[0]
    r = int(ok[0]) if len(ok) else len(rows)
    b = Y[piv[:r]]
    _, piv2 = sla.qr(M.T, mode="r", pivoting=True)
    a = X[piv2[:r]]
    D = np.linalg.pinv(green(X, b), rcond=1e-15) @ M @ np.linalg.pinv(green(a, Y), rcond=1e-15)
    return Skeleton(a=a, b=b, D=D, X=X)


def build_opset(tau: float, w_hi: int, seed: int = 12345, verbose: bool = False) -> OpSet:
    """Skeletons for widths w_hi, w_hi/2, ..., 1 (every direction) and the LF level."""
    hf = {}
    w = w_hi
    while w >= 1:
        offs = region_offsets(w)
        dirs = np.array([direction(n, w) for n in offs.tolist()])
        sk = []
        for l in range(6 * w * w):
            rng = np.random.default_rng([seed, w, l])
            own = offs[dirs == l] * float(w)
            n_own, n_y = sample_sizes(w, tau)
            parts = [_sample_boxes(rng, own, float(w), n_own)] if len(own) else []
            if 2 * w in hf:
                dl = child_deltas(float(w))
                for lp, s in enumerate(hf[2 * w]):
                    if direction_down(lp, 2 * w) == l:
                        parts.append((s.a[None, :, :] - dl[:, None, :]).reshape(-1, 3))
            X = np.concatenate(parts, axis=0)
            Y = (rng.random((n_y, 3)) - 0.5) * w
            sk.append(skeleton(X, Y, tau))
            if verbose:
                print(f"w={w} l={l} |X|={len(X)} r={sk[-1].r}", flush=True)
        hf[w] = sk
        w //= 2
    # low-frequency level, width 1/2
    rng = np.random.default_rng([seed, 0, 0])
    offs = region_offsets(0.5) * 0.5
    n_own, n_y = sample_sizes(0.5, tau)
    parts = [_sample_boxes(rng, offs, 0.5, n_own)]
    if 1 in hf:
        dl = child_deltas(0.5)
        for s in hf[1]:
            parts.append((s.a[None, :, :] - dl[:, None, :]).reshape(-1, 3))
    X = np.concatenate(parts, axis=0)
    Y = (rng.random((n_y, 3)) - 0.5) * 0.5
    lf = skeleton(X, Y, tau)
    if verbose:
        print(f"LF |X|={len(X)} r={lf.r}", flush=True)
    return OpSet(tau=tau, w_hi=w_hi, hf=hf, lf=lf)


def heldout_error(sk: Skeleton, X: np.ndarray, Y: np.ndarray) -> float:
    """||G(X,Y) - G(X,b) D G(a,Y)||_F / ||G(X,Y)||_F on fresh samples (Eq. 2 check)."""
    M = green(X, Y)
    A = green(X, sk.b) @ (sk.D @ green(sk.a, Y))
    return float(np.linalg.norm(M - A) / np.linalg.norm(M))
