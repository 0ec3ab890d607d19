"""Seeded ray batches and pixel subsets (inputs only).

`random_rays` draws arbitrary rays for testing the per-ray renderer directly:
origins on a sphere around the scene box, unit directions aimed at points in a
slightly enlarged box so that a share of rays misses, plus a few axis-aligned
and inside-the-box rays.  Pixel subsets are index arrays; turning a pixel into
a ray is the renderer's job (and the oracle's).
"""
import numpy as np


def random_rays(n, seed=5, radius=4.0, aim_half=1.9, n_axis=8, n_inside=8):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    o = radius * v
    tgt = rng.uniform(-aim_half, aim_half, size=(n, 3))
    d = tgt - o
    # axis-aligned rays (exercise zero direction components in the slab test)
    k = min(n_axis, n)
    for i in range(k):
        ax = i % 3
        sgn = 1.0 if (i // 3) % 2 == 0 else -1.0
        o[i] = rng.uniform(-1.2, 1.2, 3)
        o[i, ax] = -sgn * radius
        d[i] = 0.0
        d[i, ax] = sgn
    # rays starting inside the box
    m = min(n_inside, n - k)
    for i in range(k, k + m):
        o[i] = rng.uniform(-1.0, 1.0, 3)
        d[i] = rng.standard_normal(3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return (np.ascontiguousarray(o.astype(np.float32)),
            np.ascontiguousarray(d.astype(np.float32)))


def pixel_subset(width, height, n, seed):
    """n distinct flat pixel indices (row-major j*W+i), sorted."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(width * height, size=n, replace=False)
    return np.sort(idx).astype(np.int64)


def training_pixels(n_views, width, height, n_rays, seed):
    """n_rays distinct (view, pixel) pairs drawn without replacement from
    n_views*width*height; returns (view int32[n], pixel int64[n])."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(n_views * width * height, size=n_rays, replace=False)
    view = (flat // (width * height)).astype(np.int32)
    pix = (flat % (width * height)).astype(np.int64)
    return view, pix
