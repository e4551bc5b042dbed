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
    true_field: np.ndarray | None     # float32 (3, n0, n1, n2): moving(x) = fixed(x + g(x)); None
                                      # where it is not formed at full size
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


def _coarse_field_at(rng, shape, spacing, max_norm, points):
    """A smooth random displacement, evaluated only at `points` ((k, 3) voxel
    coordinates): N(0,1) on a coarse grid of the given spacing, smoothed there,
    interpolated with SciPy's order-1 spline, and scaled so that the largest
    displacement over the coarse grid is max_norm."""
    coarse = tuple(int(np.ceil((n - 1) / spacing)) + 1 for n in shape)
    comps = [ndi.gaussian_filter(rng.standard_normal(coarse), 1.0, mode="reflect") for _ in range(3)]
    scale = max_norm / np.sqrt(sum(c * c for c in comps)).max()
    q = (np.asarray(points, np.float64) / spacing).T
    return np.stack([scale * ndi.map_coordinates(c, q, order=1, mode="nearest") for c in comps], 1)


def _stamp(vol, centre, cov_inv, amp, half):
    """Adds amp * exp(-q^T C^-1 q / 2) on the box of half-width `half` around
    `centre` (clipped to the volume)."""
    lo = [max(0, int(np.floor(centre[k])) - half) for k in range(3)]
    hi = [min(vol.shape[k], int(np.floor(centre[k])) + half + 1) for k in range(3)]
    if any(h <= l for l, h in zip(lo, hi)):
        return
    q0, q1, q2 = (np.arange(lo[k], hi[k], dtype=np.float32) - np.float32(centre[k]) for k in range(3))
    q0, q1, q2 = q0[:, None, None], q1[None, :, None], q2[None, None, :]
    C = np.asarray(cov_inv, np.float32)
    # the quadratic form, with the broadcast axes kept separate until the sum
    e = (C[0, 0] * q0 * q0 + (2 * C[0, 1]) * q0 * q1) + ((2 * C[0, 2]) * q0 * q2 + C[1, 1] * q1 * q1) + \
        ((2 * C[1, 2]) * q1 * q2 + C[2, 2] * q2 * q2)
    vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += np.float32(amp) * np.exp(np.float32(-0.5) * e)


def microscopy_pair(shape=(512, 512, 512), seed=5, n_blobs=400, n_tubes=60, sigma_range=(2.0, 12.0),
                    tube_radius=(1.5, 4.0), photons=100.0, field_max=20.0, name="microscopy"):
    """Expansion-microscopy-like volume: anisotropic Gaussian blobs (per-axis
    sigma in sigma_range, random orientation) and tubes along smoothed random
    walks (Gaussian cross-section), with Poisson-like shot noise of variance
    I / k (k photons per unit intensity).
    The moving volume is the same scene with every structure displaced by a
    smooth random field (max field_max voxels) evaluated where it lies: a
    deformation of the scene, made without resampling the full volume, so the
    pair stays cheap to generate at 512^3 (the field itself is not formed at
    full size: true_field is None)."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    field_rng = np.random.default_rng(seed + 2)
    scene = []
    for _ in range(n_blobs):
        c = rng.uniform(0.0, 1.0, 3) * (np.array(shape) - 1)
        sig = rng.uniform(*sigma_range, size=3)
        Q, _r = np.linalg.qr(rng.standard_normal((3, 3)))
        cov_inv = Q @ np.diag(1.0 / sig ** 2) @ Q.T
        scene.append((c, cov_inv, rng.uniform(0.2, 1.0), int(np.ceil(3.0 * sig.max()))))
    for _ in range(n_tubes):
        steps = rng.normal(0.0, 8.0, size=(50, 3))
        pts = rng.uniform(0.0, 1.0, 3) * (np.array(shape) - 1) + np.cumsum(steps, axis=0)
        pts = ndi.gaussian_filter1d(pts, 5.0, axis=0, mode="nearest")
        r = rng.uniform(*tube_radius)
        amp = rng.uniform(0.3, 1.0)
        seg = np.linalg.norm(np.diff(pts, axis=0), axis=1)
        t = np.concatenate([[0.0], np.cumsum(seg)])
        sample = np.arange(0.0, t[-1], r)
        cur = np.stack([np.interp(sample, t, pts[:, k]) for k in range(3)], 1)
        cov_inv = np.eye(3) / (r * r)
        for c in cur:
            scene.append((c, cov_inv, amp * 0.4, int(np.ceil(3.0 * r))))
    # the structure at y appears at y - g(y) in the moving volume, so that
    # moving(x) = fixed(x + g(x)) to first order; g is formed only where needed
    g = _coarse_field_at(field_rng, shape, 32, field_max, np.array([c for c, _, _, _ in scene]))
    fixed = np.zeros(shape, np.float32)
    moving = np.zeros(shape, np.float32)
    for (c, cov_inv, amp, half), gc in zip(scene, g):
        _stamp(fixed, c, cov_inv, amp, half)
        _stamp(moving, c - gc, cov_inv, amp, half)
    noise = np.random.default_rng(seed + 1)
    for vol in (fixed, moving):
        # shot noise of `photons` counts per unit intensity, in its Gaussian
        # form (variance I / photons), clipped at zero
        np.clip(vol, 0.0, None, out=vol)
        vol += np.sqrt(vol / np.float32(photons)) * noise.standard_normal(shape, dtype=np.float32)
        np.clip(vol, 0.0, None, out=vol)
    return SynthPair(name, fixed, moving, None)


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


def microscopy128():
    """128^3 microscopy-like pair, four levels (8x, 4x, 2x, 1x) at 40/20/10/5
    iterations, LNCC 7^3: the 512^3 recipe's structure at a size the FP64
    oracle runs in minutes."""
    p = microscopy_pair((128, 128, 128), seed=5, n_blobs=60, n_tubes=8)
    p.name, p.scales, p.iters, p.window = "microscopy128", [8.0, 4.0, 2.0, 1.0], [40, 20, 10, 5], 7
    return p


WORKLOADS = {"blobs64": blobs64, "tissue160": tissue160, "blobs128": blobs128, "microscopy128": microscopy128}


def load(name: str, cache_dir: str | None = None) -> SynthPair:
    """Generate (or load from an .npz cache) a named workload."""
    gen = WORKLOADS[name]
    cache_dir = cache_dir or os.environ.get("FA_SYNTH_CACHE", "/tmp/fa_synth_cache")
    path = os.path.join(cache_dir, f"{name}.v1.npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            p = SynthPair(name, z["fixed"], z["moving"], z["true_field"] if "true_field" in z else None,
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
        arrays = dict(fixed=p.fixed, moving=p.moving)
        if p.true_field is not None:
            arrays["true_field"] = p.true_field
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
    "microscopy128": ([8.0, 4.0, 2.0, 1.0], [40, 20, 10, 5], 7),
}
