"""Seeded synthetic uint8 HxWx3 images.

The paper measures on ImageNet/CIFAR10 images, which are not available here.
These images stand in for them: smooth random fields with a few sharp step
edges, so that a local model sees both smooth regions and discontinuities.

Recipe G(sigma, n_edges, noise, H, W, seed):
  1. rng = numpy PCG64(seed)
  2. z ~ N(0,1), shape (H, W, 3), float64, independent per channel
  3. separable Gaussian blur, std sigma px, radius ceil(4 sigma), reflect border
  4. n_edges step edges: a line through a uniform point at a uniform angle in
     [0, pi); on its positive side add a per-channel amplitude
     U(-2, 2) * std(blurred)
  5. rescale per image to [0, 255] by (f - min) / (max - min) * 255
  6. optional integer noise U{-noise..noise} per value
  7. round half to even, clip to [0, 255], uint8
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import gaussian_filter1d


def smooth_field_image(sigma: float, n_edges: int, noise: int, H: int, W: int,
                       seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((H, W, 3))
    radius = int(math.ceil(4.0 * sigma))
    f = gaussian_filter1d(z, sigma, axis=0, mode="reflect", truncate=radius / sigma)
    f = gaussian_filter1d(f, sigma, axis=1, mode="reflect", truncate=radius / sigma)
    sd = float(f.std())
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    for _ in range(n_edges):
        py = rng.uniform(0.0, H)
        px = rng.uniform(0.0, W)
        ang = rng.uniform(0.0, math.pi)
        amp = rng.uniform(-2.0, 2.0, size=3) * sd
        side = ((xx - px) * math.cos(ang) + (yy - py) * math.sin(ang)) > 0.0
        f = f + side[:, :, None] * amp[None, None, :]
    lo, hi = float(f.min()), float(f.max())
    f = (f - lo) / (hi - lo if hi > lo else 1.0) * 255.0
    if noise:
        f = f + rng.integers(-noise, noise + 1, size=f.shape)
    return np.clip(np.rint(f), 0, 255).astype(np.uint8)


# Workloads: (description, list of (H, W), generator args (sigma, n_edges, noise), seed base)
_SIZES3 = [(64, 64), (96, 128), (256, 256), (200, 320)]


def _uneven_sizes(n: int = 64, seed: int = 3_999_999):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, len(_SIZES3), size=n)
    return [_SIZES3[int(i)] for i in idx]


WORKLOADS = {
    # one 32x32 image
    "single32": dict(shapes=[(32, 32)], gen=(2.0, 3, 0), seed_base=1_000_000),
    # 512 images of 32x32
    "batch512x32": dict(shapes=[(32, 32)] * 512, gen=(2.0, 3, 0), seed_base=2_000_000),
    # 64 images of uneven sizes
    "uneven64": dict(shapes=None, gen=(2.0, 3, 0), seed_base=3_000_000),
    # 4 x 1024^2 + 2 x 2048x1536 (H x W)
    "large6": dict(shapes=[(1024, 1024)] * 4 + [(2048, 1536)] * 2, gen=(4.0, 20, 3),
                   seed_base=4_000_000),
}


def workload_shapes(name: str):
    w = WORKLOADS[name]
    return _uneven_sizes() if w["shapes"] is None else list(w["shapes"])


def workload_images(name: str, count: int | None = None, start: int = 0):
    """Images of a named workload; `count`/`start` select a sub-range."""
    w = WORKLOADS[name]
    shapes = workload_shapes(name)
    stop = len(shapes) if count is None else min(len(shapes), start + count)
    sigma, n_edges, noise = w["gen"]
    return [smooth_field_image(sigma, n_edges, noise, H, W, w["seed_base"] + n)
            for n, (H, W) in enumerate(shapes[start:stop], start=start)]


def training_pool(n: int = 512, side: int = 64, seed_base: int = 5_000_000):
    """Pool of training images (smooth fields, sigma=2, 3 edges)."""
    return np.stack([smooth_field_image(2.0, 3, 0, side, side, seed_base + k) for k in range(n)])


def training_crops(pool: np.ndarray, batch: int, crop: int, rng: np.random.Generator):
    """`batch` random crop x crop windows from a pool of images (N, H, W, 3)."""
    N, H, W, _ = pool.shape
    ii = rng.integers(0, N, size=batch)
    yy = rng.integers(0, H - crop + 1, size=batch)
    xx = rng.integers(0, W - crop + 1, size=batch)
    return np.stack([pool[i, y:y + crop, x:x + crop] for i, y, x in zip(ii, yy, xx)])
