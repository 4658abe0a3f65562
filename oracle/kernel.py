"""Helmholtz kernel and the direct O(N^2) sum of Eq. (1) (Section 1).

Test infrastructure: imported only by tests, the smoke check and the
benchmark's CPU-baseline leg.

G(x, y) = exp(2 pi i |x - y|) / |x - y|: wavelength one, no 1/(4 pi) factor,
exactly as the paper scales the problem (Section 1, Eq. 1).  The sum in Eq. 1
runs over all j, where G is singular at j = i; the reading used here skips
every pair at distance zero (the term is defined as 0).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def green(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Matrix G[i, j] = G(x_i, y_j) for point arrays x (m, 3) and y (n, 3).

    Coincident points give 0 (reading of the j = i term of Eq. 1).
    """
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    d = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
    out = np.zeros(r.shape, dtype=np.complex128)
    nz = r > 0
    rn = r[nz]
    out[nz] = np.exp(1j * TWO_PI * rn) / rn
    return out


def direct_sum(points: np.ndarray, f: np.ndarray, targets=None, chunk: int = 32) -> np.ndarray:
    """Potentials u_i = sum_{j, p_j != p_i} G(p_i, p_j) f_j  (Eq. 1).

    points: (N, 3) float64.  f: (nrhs, N) or (N,) complex.  targets: optional
    index array; the result has shape (nrhs, len(targets)) (or (len,) for 1-D f).
    Evaluated in complex128, a block of targets at a time.
    """
    points = np.asarray(points, dtype=np.float64)
    f = np.asarray(f)
    one = f.ndim == 1
    F = np.atleast_2d(f).astype(np.complex128)
    idx = np.arange(points.shape[0]) if targets is None else np.asarray(targets)
    out = np.empty((F.shape[0], idx.size), dtype=np.complex128)
    FT = F.T.copy()
    for s in range(0, idx.size, chunk):
        t = idx[s:s + chunk]
        out[:, s:s + chunk] = (green(points[t], points) @ FT).T
    return out[0] if one else out


def rel_l2(u: np.ndarray, ref: np.ndarray) -> float:
    """Relative L2 (Frobenius) error ||u - ref|| / ||ref|| over all entries."""
    u = np.asarray(u, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
