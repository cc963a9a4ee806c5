"""Seeded synthetic inputs for the k-d tree build (shared by tests, oracle runs
and the GPU benchmark).

This module only draws numbers: it contains none of the build's arithmetic.
Every generator uses numpy's PCG64 with an explicit seed.  The paper's own
experiments use randomly generated integers (Sec. 2.3, Sec. 4, Appendix
"Performance Measurements"); the five named workloads below follow that and
add clustered, point-cloud and heavy-tailed mixtures of the same shapes.

Duplicates are planted exactly: draw ``n - d`` base rows, draw ``d`` copies
with replacement from the base rows, concatenate and shuffle the rows.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 14105420


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _plant_duplicates(g: np.random.Generator, base: np.ndarray, n: int) -> np.ndarray:
    d = n - base.shape[0]
    if d > 0:
        pick = g.integers(0, base.shape[0], size=d)
        base = np.concatenate([base, base[pick]], axis=0)
    order = g.permutation(n)
    return np.ascontiguousarray(base[order])


def uniform_int(n: int, k: int, lo: int, hi: int, dup_frac: float, seed: int) -> np.ndarray:
    """int32 rows uniform in [lo, hi) with round(dup_frac * n) planted copies."""
    g = rng(seed)
    d = int(round(dup_frac * n)) if n > 1 else 0
    d = min(d, max(n - 1, 0))
    base = g.integers(lo, hi, size=(n - d, k), dtype=np.int64).astype(np.int32)
    return _plant_duplicates(g, base, n)


def clustered_int(n: int, k: int, clusters: int, sigma: float, centre_hi: int, dup_frac: float,
                  seed: int) -> np.ndarray:
    """int32 rows from ``clusters`` isotropic Gaussians (std ``sigma``) whose
    centres are uniform in [0, centre_hi)^k, rounded to integers."""
    g = rng(seed)
    d = int(round(dup_frac * n)) if n > 1 else 0
    d = min(d, max(n - 1, 0))
    centres = g.uniform(0, centre_hi, size=(clusters, k))
    which = g.integers(0, clusters, size=n - d)
    pts = np.rint(centres[which] + g.normal(0.0, sigma, size=(n - d, k)))
    pts = np.clip(pts, -(2 ** 31), 2 ** 31 - 1).astype(np.int64).astype(np.int32)
    return _plant_duplicates(g, pts, n)


def _orthonormal_pair(g: np.random.Generator):
    a = g.normal(size=3)
    a /= np.linalg.norm(a)
    b = g.normal(size=3)
    b -= a * np.dot(a, b)
    b /= np.linalg.norm(b)
    return a, b


def point_cloud(n: int, g: np.random.Generator) -> np.ndarray:
    """float32 (n, 3) samples from 1-4 random surfaces (spheres and plane
    patches) with N(0, 1e-3) noise per coordinate."""
    surfaces = int(g.integers(1, 5))
    counts = np.bincount(g.integers(0, surfaces, size=n), minlength=surfaces)
    parts = []
    for c in counts:
        if c == 0:
            continue
        if g.random() < 0.5:
            centre = g.uniform(-10, 10, size=3)
            radius = math.exp(g.uniform(math.log(0.1), math.log(5.0)))
            v = g.normal(size=(c, 3))
            v /= np.linalg.norm(v, axis=1, keepdims=True)
            parts.append(centre + radius * v)
        else:
            origin = g.uniform(-10, 10, size=3)
            u, w = _orthonormal_pair(g)
            eu, ew = g.uniform(0.5, 5.0, size=2)
            a = g.uniform(0, eu, size=(c, 1))
            b = g.uniform(0, ew, size=(c, 1))
            parts.append(origin + a * u + b * w)
    pts = np.concatenate(parts, axis=0)
    pts = pts + g.normal(0.0, 1e-3, size=pts.shape)
    return pts.astype(np.float32)


def gaussian_mixture_f32(n: int, k: int, components: int, seed: int, log_sigma: float = 1.5,
                         mean_range: float = 100.0, sample_seed: int | None = None) -> np.ndarray:
    """float32 rows from ``components`` equal-weight anisotropic Gaussians:
    means uniform in [-mean_range, mean_range]^k, per-axis scales
    exp(N(0, log_sigma)), a random rotation per component.  The components
    come from ``seed``; the rows from the same generator, or from
    ``sample_seed`` when given (another draw of the same distribution)."""
    g = rng(seed)
    means = g.uniform(-mean_range, mean_range, size=(components, k))
    scales = np.exp(g.normal(0.0, log_sigma, size=(components, k)))
    rots = []
    for _ in range(components):
        q, r = np.linalg.qr(g.normal(size=(k, k)))
        rots.append(q * np.sign(np.diag(r)))
    rots = np.stack(rots)
    if sample_seed is not None:
        g = rng(sample_seed)
    which = g.integers(0, components, size=n)
    out = np.empty((n, k), dtype=np.float32)
    chunk = 1 << 22
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        w = which[s:e]
        z = g.standard_normal(size=(e - s, k), dtype=np.float32) * scales.astype(np.float32)[w]
        r32 = rots.astype(np.float32)
        for i in range(k):
            acc = means.astype(np.float32)[w, i]
            for j in range(k):
                acc += r32[:, i, j][w] * z[:, j]
            out[s:e, i] = acc
    return out


# ---- the five named workloads ------------------------------------------------

def c1_small_uniform() -> np.ndarray:
    """k=3, n=4096, int32 uniform in [0, 2^20), 2% exact copies."""
    return uniform_int(4096, 3, 0, 1 << 20, 0.02, SEED_BASE + 1)


def c2_full_range(n: int = 1 << 24) -> np.ndarray:
    """k=3, n=2^24, int32 uniform over the full signed range, 0.1% copies."""
    return uniform_int(n, 3, -(2 ** 31), 2 ** 31, 0.001, SEED_BASE + 2)


def c3_clustered(k: int, n: int = 1 << 22) -> np.ndarray:
    """k in {2,3,4,6,8}, n=2^22, 256 Gaussian clusters (sigma 2^12, centres
    uniform in [0, 2^30)), 10% exact copies."""
    return clustered_int(n, k, 256, float(1 << 12), 1 << 30, 0.10, SEED_BASE + 3 + 100 * k)


def c4_batched(trees: int = 4096, lo: int = 64, hi: int = 65536, seed: int = SEED_BASE + 4):
    """``trees`` point-cloud trees with log-uniform sizes in [lo, hi].

    Returns ``(tuples float32[N, 3], offsets int64[trees + 1])``.
    """
    g = rng(seed)
    sizes = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=trees))).astype(np.int64)
    sizes = np.clip(sizes, lo, hi)
    offsets = np.zeros(trees + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    parts = [point_cloud(int(s), g) for s in sizes]
    return np.ascontiguousarray(np.concatenate(parts, axis=0)), offsets


def c5_mixture(n: int = 1 << 26, draw: int = 0) -> np.ndarray:
    """k=3, n=2^26, float32 mixture of 64 anisotropic Gaussians with lognormal
    scales (mu 0, sigma 1.5).  draw > 0: another sample of the same mixture
    (same components, rows from seed SEED_BASE + 5 + 1000 * draw)."""
    if draw == 0:
        return gaussian_mixture_f32(n, 3, 64, SEED_BASE + 5)
    return gaussian_mixture_f32(n, 3, 64, SEED_BASE + 5, sample_seed=SEED_BASE + 5 + 1000 * draw)


def c2_queries(t: np.ndarray, nq: int = 1 << 20, seed: int = SEED_BASE + 6):
    """Queries over the C2 tree: ``nq`` points, each a random tuple moved by
    up to 1000 in every coordinate (nearest-neighbour queries), and ``nq``
    boxes of half-width 2^26 around random tuples (about 500 of the 2^24
    rows inside each).  Returns ``(points, lower, upper)``, int32 (nq, k)."""
    g = rng(seed)
    n, k = t.shape
    base = t[g.integers(0, n, size=nq)].astype(np.int64)
    pts = np.clip(base + g.integers(-1000, 1001, size=base.shape), -2**31, 2**31 - 1)
    centre = t[g.integers(0, n, size=nq)].astype(np.int64)
    half = 1 << 26
    lower = np.clip(centre - half, -2**31, 2**31 - 1)
    upper = np.clip(centre + half, -2**31, 2**31 - 1)
    return pts.astype(np.int32), lower.astype(np.int32), upper.astype(np.int32)
