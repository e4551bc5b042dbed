"""FP64 CPU oracle of the post hoc inverse of a FireANTs warp (arXiv 2404.01249).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library; it builds on the registration oracle (``fireants64``) for
trilinear sampling, Gaussian smoothing, Adam, the step normalisation, the
composition and the pyramid.

The paper (Section 4.4.3, "Alternative formulations for Eulerian
differential") computes phi^{-1} after the registration, by minimising
sum_x |psi(phi(x)) - x|^2 + |phi(psi(x)) - x|^2 over diffeomorphisms psi with
a multi-scale objective like the image-matching one, and uses the same
routine for the final transform of its symmetric registration.

Readings (the paper gives only the objective):

* psi = id + e and phi = id + d on the voxel grid of a level; e and d are
  sampled trilinearly with zero extension outside the grid, as everywhere in
  the registration oracle.  The two residuals are
  r1(x) = psi(phi(x)) - x = d(x) + e(x + d(x)) and
  r2(x) = phi(psi(x)) - x = e(x) + d(x + e(x)).
* The cost of a level is their mean squared norm, U = (|r1|^2 + |r2|^2) / N,
  so its scale does not depend on the level's size.
* It is minimised by Algorithm 1's own loop with U in place of the image
  cost: Gateaux gradient -> Adam -> smooth (sigma_grad) -> normalise
  (eta / (2 max |s|)) -> compose psi o (id + u) -> smooth (sigma_warp); the
  pyramid and the level transitions (e scaled by rho, Adam moments unscaled)
  are the registration's, the step count carries across levels, and psi starts
  at the identity.
* phi at a coarse level is the registration's field carried to that grid like
  an image (blur with sigma = s/2, corner-aligned trilinear resampling), each
  component divided by rho_a = (nf_a - 1)/(nc_a - 1) because voxel units grow
  with the grid spacing.

Parity status of every function is pinned in tests/test_oracle_inverse.py.
"""
from __future__ import annotations

import numpy as np

from . import fireants64 as F

__all__ = ["splat", "inverse_residuals", "inverse_cost", "inverse_gradient", "downsample_field",
           "inverse_iterate", "invert"]


def splat(vals, p, shape):
    """Adjoint of trilinear sampling in the sampled volume.

    out[j] = sum_x vals(x) w_j(p(x)), where w_j(p) is the trilinear weight of
    grid node j at position p (p has shape (3, ...) in voxel-index
    coordinates).  Nodes outside the grid receive nothing, which is the
    adjoint of the zero extension of :func:`fireants64.trilinear`.
    """
    vals = np.asarray(vals, np.float64)
    p = np.asarray(p, np.float64)
    q = np.floor(p)
    t = p - q
    q = q.astype(np.int64)
    out = np.zeros(shape)
    for b0 in (0, 1):
        for b1 in (0, 1):
            for b2 in (0, 1):
                i = (q[0] + b0, q[1] + b1, q[2] + b2)
                w = ((t[0] if b0 else 1.0 - t[0]) * (t[1] if b1 else 1.0 - t[1]) *
                     (t[2] if b2 else 1.0 - t[2]))
                ok = np.ones(vals.shape, bool)
                for a in range(3):
                    ok &= (i[a] >= 0) & (i[a] < shape[a])
                np.add.at(out, (i[0][ok], i[1][ok], i[2][ok]), (w * vals)[ok])
    return out


def _sample_field(f, p):
    return np.stack([F.trilinear(f[c], p) for c in range(3)])


def inverse_residuals(d, e):
    """(r1, r2, q, p): r1 = d + e(q) at q = x + d(x), the residual of
    psi o phi; r2 = e + d(p) at p = x + e(x), the residual of phi o psi."""
    d = np.asarray(d, np.float64)
    e = np.asarray(e, np.float64)
    X = F.identity_grid(d.shape[1:])
    q = X + d
    p = X + e
    r1 = d + _sample_field(e, q)
    r2 = e + _sample_field(d, p)
    return r1, r2, q, p


def inverse_cost(d, e):
    """U(e) = (sum |psi(phi(x)) - x|^2 + |phi(psi(x)) - x|^2) / N."""
    r1, r2, _, _ = inverse_residuals(d, e)
    return float(((r1 * r1).sum() + (r2 * r2).sum()) / r1[0].size)


def inverse_gradient(d, e):
    """(g, U): dU/de at every grid node, and U.

    The first sum reaches e through its samples at q(x): its derivative is
    the splat of 2 r1 at q.  The second reaches e(x) directly and through
    d(x + e(x)): 2 (I + grad d(p))^T r2, with grad d the derivative of the
    trilinear sample (from the right at integer coordinates).
    """
    d = np.asarray(d, np.float64)
    shape = d.shape[1:]
    r1, r2, q, p = inverse_residuals(d, e)
    N = float(np.prod(shape))
    g = np.stack([2.0 * splat(r1[c], q, shape) for c in range(3)])
    Jd = np.stack([F.trilinear_dpos(d[c], p) for c in range(3)])   # Jd[c, a] = d d_c / d p_a
    for a in range(3):
        g[a] += 2.0 * (r2[a] + sum(Jd[c, a] * r2[c] for c in range(3)))
    U = ((r1 * r1).sum() + (r2 * r2).sum()) / N
    return g / N, float(U)


def downsample_field(d, scale):
    """The warp's field at downsampling factor ``scale``: each component
    blurred (sigma = scale/2) and resampled at corner-aligned positions like
    an image, then divided by rho_a = (nf_a - 1)/(nc_a - 1).  Identity at
    scale 1."""
    d = np.asarray(d, np.float64)
    shp_f = d.shape[1:]
    shp_c = F.level_shape(shp_f, scale)
    if float(np.float32(scale)) == 1.0 and shp_c == shp_f:
        return d.copy()
    rho = [((shp_f[a] - 1) / (shp_c[a] - 1)) if shp_c[a] > 1 else 1.0 for a in range(3)]
    pos = F._aligned_positions(shp_f, shp_c)
    s = float(np.float32(scale)) / 2.0
    return np.stack([F.trilinear(F.gaussian_smooth(d[c], s), pos) / rho[c] for c in range(3)])


def inverse_iterate(d, e, m, v, t, P: F.Params):
    """One iteration of Algorithm 1 on the inverse's cost (psi = id + e)."""
    g, U = inverse_gradient(d, e)
    a, m, v = F.adam_update(g, m, v, t, P.beta1, P.beta2, P.adam_eps)
    s = F.gaussian_smooth(a, P.sigma_grad)
    u, M = F.normalise_step(s, P.eta)
    e1 = F.compose(e, u)
    e_new = F.gaussian_smooth(e1, P.sigma_warp)
    return e_new, m, v, U, dict(g=g, a=a, s=s, M=M, u=u, e_composed=e1)


def invert(d, scales, iters, P: F.Params, callback=None):
    """psi = phi^{-1} fitted over the pyramid.  Returns (e, losses, t): the
    inverse's displacement at the finest level, one cost per iteration (before
    that iteration's update) and the final step count."""
    d = np.asarray(d, np.float64)
    e = m = v = None
    t = 0
    losses = []
    for lvl, (s, T) in enumerate(zip(scales, iters)):
        dl = downsample_field(d, s)
        if e is None:
            e = np.zeros_like(dl)
            m = np.zeros_like(dl)
            v = np.zeros_like(dl)
        else:
            e, m, v = F.upsample_state(e, m, v, dl.shape[1:])
        for i in range(int(T)):
            t += 1
            e, m, v, U, ex = inverse_iterate(dl, e, m, v, t, P)
            losses.append(U)
            if callback is not None:
                callback(lvl, i, e, m, v, U, ex)
    return e, losses, t
