"""Seeded synthetic inputs for the directional FMM matvec.

This module only draws points and densities; it holds none of the method's
arithmetic, so both the CPU oracle (``oracle/``) and the GPU path may use it.

The paper (Section 4.2) samples points randomly on triangulated surfaces
(sphere, F16, submarine) and draws densities from a standard normal
distribution.  The aircraft and submarine meshes are not available, so the
surfaces here are analytic stand-ins: spheres, an area-uniform ellipsoid and a
union of non-overlapping spheres, all inside the ball |p| <= K/2 of Eq. (1).

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and returns
float64 points of shape (N, 3), row-major (x, y, z), in wavelengths.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sphere_points",
    "ellipsoid_points",
    "sphere_union_points",
    "densities",
    "sample_targets",
    "CONFIGS",
    "make_config",
    "SERVING_PLANS",
    "serving_points",
    "serving_mix",
]


def sphere_points(n: int, K: float, seed: int) -> np.ndarray:
    """N points uniform on the sphere of diameter K centred at the origin."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return (K / 2.0) * g / np.linalg.norm(g, axis=1, keepdims=True)


def ellipsoid_points(n: int, semi_axes, seed: int) -> np.ndarray:
    """N points on the ellipsoid with the given semi-axes, density uniform in area.

    Rejection sampling on the unit sphere: a direction u is kept with
    probability g(u)/g_max where g(u) = sqrt(sum u_k^2 / s_k^2) is the area
    element of the map u -> (s_1 u_1, s_2 u_2, s_3 u_3) up to a constant, and
    g_max = 1/min(s).  Batches of 2N candidates are drawn until N are kept;
    the first N kept, in draw order, are returned.
    """
    a, b, c = (float(s) for s in semi_axes)
    rng = np.random.default_rng(seed)
    s = np.array([a, b, c])
    gmax = 1.0 / s.min()
    out = []
    kept = 0
    while kept < n:
        u = rng.standard_normal((2 * n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = rng.random(2 * n)
        g = np.sqrt(np.sum((u / s) ** 2, axis=1))
        sel = u[r < g / gmax]
        out.append(sel * s)
        kept += len(sel)
    return np.concatenate(out, axis=0)[:n]


def sphere_union_points(n: int, K: float, n_spheres: int, seed: int) -> np.ndarray:
    """Union of ``n_spheres`` non-overlapping spheres of diameter K/4 inside |p| <= K/2.

    Centres are drawn uniformly in the cube [-3K/8, 3K/8]^3 by rejection so
    that |c| + K/8 <= K/2 and pairwise distances are at least K/4; each sphere
    carries n // n_spheres points (the last one takes the remainder).
    """
    rng = np.random.default_rng(seed)
    rad = K / 8.0
    centres = []
    while len(centres) < n_spheres:
        c = rng.uniform(-3 * K / 8, 3 * K / 8, size=3)
        if np.linalg.norm(c) + rad > K / 2:
            continue
        if any(np.linalg.norm(c - d) < 2 * rad for d in centres):
            continue
        centres.append(c)
    counts = [n // n_spheres] * n_spheres
    counts[-1] += n - sum(counts)
    pts = []
    for c, m in zip(centres, counts):
        g = rng.standard_normal((m, 3))
        pts.append(c + rad * g / np.linalg.norm(g, axis=1, keepdims=True))
    return np.concatenate(pts, axis=0)


def densities(n: int, nrhs: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex densities of shape (nrhs, N): real and imaginary parts iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nrhs, n, 2))
    return (z[..., 0] + 1j * z[..., 1]).astype(dtype)


def sample_targets(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct target indices drawn uniformly without replacement, sorted."""
    if m >= n:
        return np.arange(n)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=m, replace=False))


# Named workloads.  ``eps`` is the end-to-end relative L2 target of the plan.
CONFIGS = {
    # sphere of diameter 4, every target checked against the direct sum
    "sphere4": dict(kind="sphere", K=4.0, N=4096, seed=1, fseed=101, nrhs=1,
                    eps=1e-6, n_check=4096, check_seed=0),
    # sphere of diameter 16, N = 65,536, one right-hand side
    "sphere16": dict(kind="sphere", K=16.0, N=65536, seed=2, fseed=202, nrhs=1,
                     eps=1e-4, n_check=2048, check_seed=202),
    # 4:2:1 ellipsoid with semi-axes (16, 8, 4) in a K = 32 box, 32 right-hand sides
    "ellipsoid32": dict(kind="ellipsoid", K=32.0, N=262144, seed=3, fseed=303,
                        nrhs=32, eps=1e-4, n_check=2048, check_seed=303),
}


def make_config(name: str, **over):
    """Return (points, f, cfg) for a named workload; keyword overrides apply to cfg."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    K, N = cfg["K"], cfg["N"]
    if cfg["kind"] == "sphere":
        pts = sphere_points(N, K, cfg["seed"])
    elif cfg["kind"] == "ellipsoid":
        pts = ellipsoid_points(N, (K / 2, K / 4, K / 8), cfg["seed"])
    elif cfg["kind"] == "union":
        pts = sphere_union_points(N, K, 8, cfg["seed"])
    else:
        raise ValueError(cfg["kind"])
    f = densities(N, cfg["nrhs"], cfg["fseed"])
    return pts, f, cfg


# The resident plans of the serving mix: (name, kind, K, N, seed).  Spheres of
# diameter K, 4:2:1 ellipsoids with semi-axes (K/2, K/4, K/8), and the union of
# 8 spheres of diameter K/4; N from 16,384 to 524,288.
SERVING_PLANS = [
    ("sphere8", "sphere", 8.0, 16384, 51),
    ("sphere16", "sphere", 16.0, 65536, 52),
    ("sphere32", "sphere", 32.0, 524288, 53),
    ("ellipsoid16", "ellipsoid", 16.0, 16384, 54),
    ("ellipsoid32", "ellipsoid", 32.0, 131072, 55),
    ("union32", "union", 32.0, 131072, 56),
]


def serving_points(kind: str, K: float, N: int, seed: int) -> np.ndarray:
    if kind == "sphere":
        return sphere_points(N, K, seed)
    if kind == "ellipsoid":
        return ellipsoid_points(N, (K / 2, K / 4, K / 8), seed)
    if kind == "union":
        return sphere_union_points(N, K, 8, seed)
    raise ValueError(kind)


def serving_mix(n: int, n_plans: int, seed: int, nrhs_choices=(1, 4, 16)):
    """A request stream: plan index uniform over n_plans, nrhs uniform over
    nrhs_choices, and unit-rate Poisson inter-arrival gaps (divide by the
    rate in requests per second for arrival times in seconds)."""
    rng = np.random.default_rng(seed)
    plan = rng.integers(0, n_plans, size=n)
    nrhs = rng.choice(np.asarray(nrhs_choices), size=n)
    gaps = rng.exponential(1.0, size=n)
    return plan, nrhs, gaps
