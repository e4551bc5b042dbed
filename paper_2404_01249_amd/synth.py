"""Seeded synthetic registration pairs.

These stand in for the paper's datasets (brain MRI of the Klein/OASIS studies,
lung CT, expansion microscopy), none of which are available here.  Each recipe
produces a fixed image, a known smooth displacement, and a moving image made by
warping the fixed image with it, so a registration has a known answer.

This module is shared input plumbing for the tests, the benchmark and the
smoke check.  It deliberately contains none of the registration method's own
arithmetic: smoothing and resampling of the synthetic volumes use SciPy's
library routines (``scipy.ndimage.gaussian_filter`` and
``scipy.ndimage.map_coordinates``), never the library or the oracle.

Every generator is a pure function of its seed.  Arrays are float32, C order,
shape ``(n0, n1, n2)`` with ``n2`` contiguous; fields are ``(3, n0, n1, n2)`` in
voxel units, component ``c`` along axis ``c``.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.ndimage as ndi


@dataclass
class SynthPair:
    """One synthetic registration problem."""
    name: str
    fixed: np.ndarray                 # float32 (n0, n1, n2)
    moving: np.ndarray                # float32 (n0, n1, n2)
    true_field: np.ndarray            # float32 (3, n0, n1, n2): moving(x) = fixed(x + g(x))
    fixed_labels: np.ndarray | None = None    # int8, classes 0..3 (label recipe only)
    moving_labels: np.ndarray | None = None
    scales: list = field(default_factory=list)
    iters: list = field(default_factory=list)
    window: int = 5


def _smooth_noise(rng, shape, sigma, truncate=3.0):
    return ndi.gaussian_filter(rng.standard_normal(shape), sigma, mode="reflect", truncate=truncate)


def _random_field(rng, shape, sigma, max_norm):
    """Three independently smoothed N(0,1) components scaled so max |g| = max_norm."""
    g = np.stack([_smooth_noise(rng, shape, sigma) for _ in range(3)])
    g *= max_norm / np.sqrt((g * g).sum(0)).max()
    return g


def _warp_linear(img, g):
    """img(x + g(x)) with SciPy's order-1 spline (= trilinear), zero outside."""
    coords = np.indices(img.shape, dtype=np.float64) + g
    return ndi.map_coordinates(img, coords, order=1, mode="constant", cval=0.0)


def _warp_nearest(lab, g):
    coords = np.indices(lab.shape, dtype=np.float64) + g
    return ndi.map_coordinates(lab, coords, order=0, mode="constant", cval=0)


def blobs_pair(shape=(64, 64, 64), seed=1, n_blobs=20, sigma_range=(4.0, 8.0),
               amp_range=(0.2, 1.0), noise_sd=0.01, field_sigma=6.0, field_max=3.0,
               name="blobs"):
    """Sum of isotropic Gaussian blobs plus white noise; moving = fixed warped by a
    smooth random field.  The defaults are the 64^3 two-level parity workload."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    grid = np.indices(shape, dtype=np.float64)
    f = np.zeros(shape)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * (np.array(shape) - 1)
    sigmas = rng.uniform(*sigma_range, size=n_blobs)
    amps = rng.uniform(*amp_range, size=n_blobs)
    for c, s, a in zip(centres, sigmas, amps):
        r2 = sum((grid[k] - c[k]) ** 2 for k in range(3))
        f += a * np.exp(-r2 / (2.0 * s * s))
    f += noise_sd * rng.standard_normal(shape)
    g = _random_field(rng, shape, field_sigma, field_max)
    mov = _warp_linear(f, g)
    return SynthPair(name, f.astype(np.float32), mov.astype(np.float32), g.astype(np.float32))


def tissue_pair(shape=(160, 192, 224), seed=2, label_sigma=4.0, bias_sigma=24.0,
                bias_amp=0.1, noise_sd=0.02, field_sigma=12.0, field_max=8.0,
                class_means=(0.1, 0.4, 0.7, 0.9), name="tissue"):
    """Brain-MRI-like volume: four piecewise-constant classes from thresholded
    smooth noise, a smooth multiplicative bias field and white noise."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    z = _smooth_noise(rng, shape, label_sigma, truncate=4.0)
    q = np.quantile(z, [0.25, 0.5, 0.75])
    labels = np.digitize(z, q).astype(np.int8)
    b = _smooth_noise(rng, shape, bias_sigma)
    b = 2.0 * (b - b.min()) / (b.max() - b.min()) - 1.0
    bias = 1.0 + bias_amp * b
    f = np.asarray(class_means)[labels] * bias + noise_sd * rng.standard_normal(shape)
    g = _random_field(rng, shape, field_sigma, field_max)
    mov = _warp_linear(f, g)
    mlab = _warp_nearest(labels.astype(np.float64), g).astype(np.int8)
    return SynthPair(name, f.astype(np.float32), mov.astype(np.float32), g.astype(np.float32),
                     fixed_labels=labels, moving_labels=mlab)


def smooth_field(shape, seed, sigma=6.0, max_norm=2.0):
    """A smooth random displacement (float32, (3,)+shape) for gradient checks."""
    rng = np.random.default_rng(seed)
    return _random_field(rng, tuple(shape), sigma, max_norm).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def blobs64():
    """64^3 blobs pair, two levels (2x, 1x) at 100/50 iterations, LNCC 5^3."""
    p = blobs_pair((64, 64, 64), seed=1)
    p.name, p.scales, p.iters, p.window = "blobs64", [2.0, 1.0], [100, 50], 5
    return p


def tissue160():
    """160x192x224 tissue pair, three levels (4x, 2x, 1x) at 200/100/50, LNCC 5^3."""
    p = tissue_pair((160, 192, 224), seed=2)
    p.name, p.scales, p.iters, p.window = "tissue160", [4.0, 2.0, 1.0], [200, 100, 50], 5
    return p


def blobs128():
    """128^3 blobs pair for gradient checks (blob widths doubled for the size)."""
    p = blobs_pair((128, 128, 128), seed=3, sigma_range=(8.0, 16.0), field_sigma=12.0)
    p.name, p.scales, p.iters, p.window = "blobs128", [1.0], [1], 5
    return p


WORKLOADS = {"blobs64": blobs64, "tissue160": tissue160, "blobs128": blobs128}


def load(name: str, cache_dir: str | None = None) -> SynthPair:
    """Generate (or load from an .npz cache) a named workload."""
    gen = WORKLOADS[name]
    cache_dir = cache_dir or os.environ.get("FA_SYNTH_CACHE", "/tmp/fa_synth_cache")
    path = os.path.join(cache_dir, f"{name}.v1.npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            p = SynthPair(name, z["fixed"], z["moving"], z["true_field"],
                          z["fixed_labels"] if "fixed_labels" in z else None,
                          z["moving_labels"] if "moving_labels" in z else None)
            meta = _META[name]
            p.scales, p.iters, p.window = list(meta[0]), list(meta[1]), meta[2]
            return p
        except Exception:  # a truncated cache file: regenerate
            pass
    p = gen()
    try:
        os.makedirs(cache_dir, exist_ok=True)
        arrays = dict(fixed=p.fixed, moving=p.moving, true_field=p.true_field)
        if p.fixed_labels is not None:
            arrays.update(fixed_labels=p.fixed_labels, moving_labels=p.moving_labels)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, **arrays)
        os.replace(tmp, path)
    except OSError:
        pass
    return p


_META = {
    "blobs64": ([2.0, 1.0], [100, 50], 5),
    "tissue160": ([4.0, 2.0, 1.0], [200, 100, 50], 5),
    "blobs128": ([1.0], [1], 5),
}
