"""FP64 CPU oracle of FireANTs' symmetric registration (arXiv 2404.01249).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library; it builds on the registration oracle (``fireants64``) and the
post hoc inverse (``inverse64``).

The paper reports a symmetric variant of its registration (Table
"timingbrain", "Ours (symmetric)") whose final transform is
phi = phi_M o phi_F^{-1}, with phi_F^{-1} from the post hoc inverse routine
(Section 4.4.3, "Alternative formulations for Eulerian differential").

Readings (the paper names the final composition only):

* The two half-way warps phi_F = id + d_F and phi_M = id + d_M minimise the
  image cost between the two warped images, C(I_F o phi_F, I_M o phi_M), so
  that the images meet in between; then I_F(x) ~ I_M(phi_M(phi_F^{-1}(x))).
* LNCC is symmetric in its two images, so dC/dd_M is the registration's
  Gateaux gradient with I_F o phi_F as the fixed image, and dC/dd_F the same
  with the roles swapped.  Both are taken at the same pair of warps (a
  simultaneous update).
* Each half-way warp is advanced by Algorithm 1's own steps with its own Adam
  moments and its own step norm M; the two share the step count, the pyramid
  and the level transitions.  Both start at the identity.
* The final field is d(x) = e(x) + d_M(x + e(x)), with psi = id + e the
  fitted inverse of phi_F.
"""
from __future__ import annotations

import numpy as np

from . import fireants64 as F
from . import inverse64 as V

__all__ = ["symmetric_cost", "symmetric_gradients", "symmetric_iterate", "register_halfway",
           "compose_fields", "register_symmetric"]


def symmetric_cost(If, Im, dF, dM, window, eps):
    """C = -mean cc(I_F o phi_F, I_M o phi_M)."""
    _, L, _ = F.lncc_forward(F.warp_image(If, dF), F.warp_image(Im, dM), window, eps)
    return float(L)


def symmetric_gradients(If, Im, dF, dM, window, eps):
    """(g_F, g_M, C): the Gateaux gradients of C with respect to d_F and d_M.

    g_M is the registration's gradient with I_F o phi_F fixed and I_M moving;
    g_F is the same with the roles swapped (cc is symmetric in its images)."""
    JF = F.warp_image(If, dF)
    JM = F.warp_image(Im, dM)
    gM, L = F.gateaux_gradient(JF, Im, dM, window, eps)
    gF, _ = F.gateaux_gradient(JM, If, dF, window, eps)
    return gF, gM, float(L)


def _advance(d, g, m, v, t, P):
    a, m, v = F.adam_update(g, m, v, t, P.beta1, P.beta2, P.adam_eps)
    s = F.gaussian_smooth(a, P.sigma_grad)
    u, _ = F.normalise_step(s, P.eta)
    return F.gaussian_smooth(F.compose(d, u), P.sigma_warp), m, v


def symmetric_iterate(If, Im, dF, dM, sF, sM, t, P: F.Params):
    """One iteration: both gradients at the current pair of warps, then each
    warp advanced by Algorithm 1's steps.  sF, sM = (m, v) of each side."""
    gF, gM, L = symmetric_gradients(If, Im, dF, dM, P.window, P.cc_eps)
    dF2, mF, vF = _advance(dF, gF, sF[0], sF[1], t, P)
    dM2, mM, vM = _advance(dM, gM, sM[0], sM[1], t, P)
    return dF2, dM2, (mF, vF), (mM, vM), L


def register_halfway(fixed, moving, scales, iters, P: F.Params):
    """The two half-way warps over the pyramid.  Returns (d_F, d_M, losses)."""
    fixed = np.asarray(fixed, np.float64)
    moving = np.asarray(moving, np.float64)
    dF = dM = None
    t = 0
    losses = []
    for s, T in zip(scales, iters):
        If = F.downsample_image(fixed, s)
        Im = F.downsample_image(moving, s)
        if dF is None:
            z = np.zeros((3,) + If.shape)
            dF, dM = z.copy(), z.copy()
            sF = (z.copy(), z.copy())
            sM = (z.copy(), z.copy())
        else:
            dF, mF, vF = F.upsample_state(dF, sF[0], sF[1], If.shape)
            dM, mM, vM = F.upsample_state(dM, sM[0], sM[1], If.shape)
            sF, sM = (mF, vF), (mM, vM)
        for _ in range(int(T)):
            t += 1
            dF, dM, sF, sM, L = symmetric_iterate(If, Im, dF, dM, sF, sM, t, P)
            losses.append(L)
    return dF, dM, losses


def compose_fields(e, dM):
    """Displacement of phi_M o psi for psi = id + e: e(x) + d_M(x + e(x))."""
    return F.compose(dM, e)


def register_symmetric(fixed, moving, scales, iters, P: F.Params, inv_scales, inv_iters, P_inv: F.Params):
    """phi = phi_M o phi_F^{-1}.  Returns (d, d_F, d_M, losses, inverse losses)."""
    dF, dM, losses = register_halfway(fixed, moving, scales, iters, P)
    e, inv_losses, _ = V.invert(dF, inv_scales, inv_iters, P_inv)
    return compose_fields(e, dM), dF, dM, losses, inv_losses
