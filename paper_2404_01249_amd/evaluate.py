"""Accuracy measures of a registration result, computed by the HIP library
(include/fa_eval.h): label transfer by nearest neighbour, per-region overlap
(target overlap and Dice / mean overlap, the paper's brain-MRI measures) and
the fraction of voxels where det(I + grad d) <= 0 (singularity error)."""
from __future__ import annotations

import numpy as np
import torch

from . import fa


def warp_labels(labels, d):
    """labels(round(x + d(x))) as int8, -1 where the position leaves the grid."""
    out = torch.empty_like(labels)
    fa.fa_warp_labels(labels, d, out)
    return out


def label_overlap(a, b, n_classes: int) -> np.ndarray:
    """(n_classes, 3) int64 counts: |a = r|, |b = r|, |a = r and b = r|."""
    return fa.fa_label_overlap(a.reshape(-1), b.reshape(-1), n_classes)


def dice(a, b, n_classes: int) -> float:
    """Mean over classes 0..n_classes-1 of 2|A_r n B_r| / (|A_r| + |B_r|)
    (1 for a class absent from both)."""
    c = label_overlap(a, b, n_classes)
    den = c[:, 0] + c[:, 1]
    per = np.where(den > 0, 2.0 * c[:, 2] / np.maximum(den, 1), 1.0)
    return float(per.mean())


def target_overlap(a, b, n_classes: int) -> float:
    """Mean over classes of |A_r n B_r| / |B_r| (b is the target)."""
    c = label_overlap(a, b, n_classes)
    per = np.where(c[:, 1] > 0, c[:, 2] / np.maximum(c[:, 1], 1), 1.0)
    return float(per.mean())


def jacobian_det(d):
    """det(I + grad d) at the interior voxels, float64 (n0-2, n1-2, n2-2)."""
    shp = tuple(max(int(n) - 2, 0) for n in d.shape[1:])
    det = torch.empty(shp, dtype=torch.float64, device=d.device)
    fa.fa_jacobian_det(d, det if det.numel() else None, count=False)
    return det


def singular_fraction(d) -> float:
    """Fraction of interior voxels with det(I + grad d) <= 0."""
    nonpos, interior = fa.fa_jacobian_det(d, None, count=True)
    return nonpos / interior if interior else float("nan")


def compose(u, d):
    """u + d(x + u) (fa_compose_fields): the displacement of (id + d) o (id + u)."""
    out = torch.empty_like(u)
    fa.fa_compose_fields(u.contiguous(), d.contiguous(), out)
    return out


def endpoint_error(d_reg, g_true, margin=8):
    """Mean and max of |d_reg(x) + g_true(x + d_reg(x))| over voxels at least
    `margin` from every face: the distance by which a registration result
    misses the warp that made the moving image (moving(x) = fixed(x + g(x)))."""
    r = compose(d_reg, g_true)
    core = (slice(None),) + tuple(slice(margin, n - margin) for n in r.shape[1:])
    e = r[core].norm(dim=0)
    return float(e.mean()), float(e.max())
