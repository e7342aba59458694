"""Seeded synthetic workloads (inputs only).

This module draws the point clouds and grids that both the GPU path and the
CPU oracle are run on.  It holds none of the reduction's arithmetic: only
random draws, the workload's threshold choice (a percentile of the pairwise
squared distances) and the smoothing that makes the grid a Gaussian random
field.  Every generator is deterministic in its seed.

Workloads (the paper's own point clouds are not available; these stand in
for them at the sizes the GPU path is measured on):

* ``vr_grid_cloud``  -- 50 points uniform on the integer grid [0,1024)^3.
* ``vr_torus``       -- 400 points on a torus (R=2, r=0.7) in R^3, area
  uniform, Gaussian noise sigma=0.05, quantised to a 2^16 grid; truncated at
  the 20th percentile of the pairwise squared distances.
* ``vr_batch``       -- 512 clouds, n ~ U{32..256}, ambient dim ~ U{2..8},
  generator ~ U{cube, noisy sphere, noisy circle}, on a 2^16 grid, each
  truncated at its own 30th percentile.
* ``circle_batch``   -- 64 clouds x 128 FP32 points on a noisy unit circle
  (sigma=0.1), full 2-skeleton.
* ``gaussian_field`` -- 64^3 white noise smoothed by a separable Gaussian
  (sigma 4 cells, periodic, truncated at 4 sigma), standardised, FP32.
"""
from __future__ import annotations

import math

import numpy as np


def percentile_threshold_sqd(pts: np.ndarray, p: float) -> int:
    """Nearest-rank p-quantile of the C(n,2) exact int64 squared distances:
    the k-th smallest with k = ceil(p * C(n,2)) (1-based)."""
    x = np.asarray(pts, np.int64)
    n = x.shape[0]
    if n < 2:
        return 0
    d = x[:, None, :] - x[None, :, :]
    sq = (d * d).sum(-1)
    iu = np.triu_indices(n, 1)
    vals = np.sort(sq[iu])
    k = max(1, int(math.ceil(p * vals.shape[0])))
    return int(vals[k - 1])


def vr_grid_cloud(seed: int = 1, n: int = 50, side: int = 1024, D: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, side, size=(n, D)).astype(np.int32)


def _quantise(y: np.ndarray, lo: float, hi: float) -> np.ndarray:
    q = np.rint((y - lo) / (hi - lo) * 65535.0)
    return np.clip(q, 0, 65535).astype(np.int32)


def vr_torus(seed: int = 2, n: int = 400, R: float = 2.0, r: float = 0.7, sigma: float = 0.05,
             pct: float = 0.20):
    """Returns (points int32 [n,3], threshold on squared distance)."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, n)
    phi = np.empty(n)
    k = 0
    while k < n:  # area-uniform tube angle by rejection
        cand = rng.uniform(0.0, 2.0 * math.pi)
        if rng.uniform(0.0, 1.0) <= (R + r * math.cos(cand)) / (R + r):
            phi[k] = cand
            k += 1
    x = np.stack([(R + r * np.cos(phi)) * np.cos(theta),
                  (R + r * np.cos(phi)) * np.sin(theta),
                  r * np.sin(phi)], axis=1)
    x = x + rng.normal(0.0, sigma, x.shape)
    pts = _quantise(x, -3.0, 3.0)
    return pts, percentile_threshold_sqd(pts, pct)


def vr_batch_instance(seq: np.random.SeedSequence, pct: float = 0.30, n_range=(32, 256),
                      d_range=(2, 8), sigma: float = 0.05):
    rng = np.random.default_rng(seq)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    D = int(rng.integers(d_range[0], d_range[1] + 1))
    kind = int(rng.integers(0, 3))
    if kind == 0:    # uniform cube
        y = rng.uniform(-1.0, 1.0, (n, D))
    elif kind == 1:  # noisy sphere S^{D-1}
        g = rng.normal(0.0, 1.0, (n, D))
        y = g / np.linalg.norm(g, axis=1, keepdims=True) + rng.normal(0.0, sigma, (n, D))
    else:            # noisy circle in the first two coordinates
        a = rng.uniform(0.0, 2.0 * math.pi, n)
        y = np.zeros((n, D))
        y[:, 0] = np.cos(a)
        y[:, 1] = np.sin(a)
        y = y + rng.normal(0.0, sigma, (n, D))
    pts = _quantise(y, -1.5, 1.5)
    return pts, percentile_threshold_sqd(pts, pct)


def vr_batch(seed: int = 3, count: int = 512, **kw):
    """List of (points int32 [n_b, D_b], threshold) for ``count`` instances."""
    return [vr_batch_instance(s, **kw) for s in np.random.SeedSequence(seed).spawn(count)]


def circle_batch(seed: int = 4, clouds: int = 64, n: int = 128, sigma: float = 0.1) -> np.ndarray:
    """FP32 [clouds, n, 2] noisy unit circles."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 2.0 * math.pi, (clouds, n))
    x = np.stack([np.cos(a), np.sin(a)], axis=-1) + rng.normal(0.0, sigma, (clouds, n, 2))
    return x.astype(np.float32)


def _gauss_kernel(sigma: float):
    h = int(math.ceil(4.0 * sigma))
    t = np.arange(-h, h + 1, dtype=np.float64)
    w = np.exp(-0.5 * (t / sigma) ** 2)
    return t.astype(np.int64), w / w.sum()


def gaussian_field(seed: int = 5, n: int = 64, sigma: float = 4.0, shape=None) -> np.ndarray:
    """FP32 [nz, ny, nx] standardised Gaussian random field (x fastest)."""
    rng = np.random.default_rng(seed)
    shp = tuple(shape) if shape is not None else (n, n, n)
    f = rng.normal(0.0, 1.0, shp)
    offs, w = _gauss_kernel(sigma)
    for ax in range(3):
        acc = np.zeros_like(f)
        for o, wt in zip(offs, w):
            acc += wt * np.roll(f, int(o), axis=ax)
        f = acc
    f = (f - f.mean()) / f.std()
    return f.astype(np.float32)


def random_grid(seed: int, shape, ties: bool = False) -> np.ndarray:
    """Small FP32 grids for parity tests; ``ties`` draws from few values."""
    rng = np.random.default_rng(seed)
    if ties:
        return rng.integers(-3, 4, size=shape).astype(np.float32)
    return rng.normal(0.0, 1.0, shape).astype(np.float32)
