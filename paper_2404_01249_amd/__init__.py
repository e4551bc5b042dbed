"""MI355X-native FireANTs dense matching step (arXiv 2404.01249).

The computation lives in the HIP library ``libfa_mi355x.so`` (C ABI in
``include/*.h``); :mod:`paper_2404_01249_amd.fa` binds it with the same
names.  Convenience wrappers over those calls:

* :class:`Pair` -- one registration (Algorithm 1), with ``autotune``;
* :func:`run_batch` -- several registrations advanced together (separate
  streams, or batched launches with optional graph replay);
* :class:`LNCC` -- the fused cost and gradient as a differentiable loss;
* :class:`Inverse` -- the post hoc inverse of a warp;
* :class:`Symmetric` -- the symmetric registration phi_M o phi_F^{-1};
* :mod:`evaluate` -- label transfer, Dice, det J, field composition.

PyTorch only provides device memory and streams.
"""
from __future__ import annotations

from . import evaluate, fa
from .fa import FAError
from .lncc import LNCC

__all__ = ["Pair", "Inverse", "Symmetric", "FAError", "fa", "LNCC", "evaluate", "run_batch"]


def run_batch(pairs, max_iters=1 << 30, fused=True, graphs=False):
    """Advance several :class:`Pair` objects together.  fused=True
    (fa_batch_step_fused): one launch per kernel for all pairs that share its
    template parameters; graphs=True replays each batch composition's
    iteration from a captured HIP graph.  fused=False (fa_batch_step): each
    pair on its own stream, interleaved.  Returns the number of pairs whose
    schedule is complete."""
    if not fused:
        return fa.fa_batch_step([p.handle for p in pairs], max_iters)
    fa.fa_batch_use_graphs(graphs)
    try:
        return fa.fa_batch_step_fused([p.handle for p in pairs], max_iters)
    finally:
        fa.fa_batch_use_graphs(False)


class Pair:
    """One registration problem: fixed and moving 3-D float32 GPU tensors.

    >>> p = Pair(fixed, moving, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
    >>> p.set_schedule([4, 2, 1], [200, 100, 50]); p.run()
    >>> d = p.field()          # (3, n0, n1, n2) displacement in voxels
    """

    def __init__(self, fixed, moving, *, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5,
                 cc_eps=1e-5, beta1=0.9, beta2=0.999, adam_eps=1e-8, use_jac=False, stream=None):
        import torch
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = fa.fa_params_default()
        p.eta, p.sigma_grad, p.sigma_warp, p.cc_window = eta, sigma_grad, sigma_warp, window
        p.cc_eps, p.adam_beta1, p.adam_beta2, p.adam_eps = cc_eps, beta1, beta2, adam_eps
        p.use_jac = 1 if use_jac else 0
        self.params = p
        self.shape = tuple(int(s) for s in fixed.shape)
        self.handle = fa.fa_pair_create(fixed, moving, p, self.stream)
        self._keep = (fixed, moving)   # alive until the stream has copied them
        self.total_iters = 0

    # -- Algorithm 1 driver -------------------------------------------------
    def set_schedule(self, scales, iters):
        fa.fa_pair_set_schedule(self.handle, scales, iters)
        self.total_iters = int(sum(iters))

    def step(self, n):
        return fa.fa_pair_step(self.handle, n)

    def autotune(self, trials=5):
        """Time candidate launch shapes per level and kernel; keep the fastest
        (after set_schedule; the state is unchanged)."""
        fa.fa_pair_autotune(self.handle, trials)

    def tiling(self, level, kind):
        """(ty, tx, zc, brick) of kernel `kind` (0 gradient, 1 sigma_grad
        smoothing, 2 sigma_warp smoothing, 3 composition) at `level`."""
        return fa.fa_pair_get_tiling(self.handle, level, kind)

    def run(self):
        done, fin = fa.fa_pair_step(self.handle, 1 << 30)
        return done

    # -- readback ---------------------------------------------------------------
    def loss_history(self):
        return fa.fa_pair_get_loss(self.handle, self.total_iters)

    def level_shape(self):
        return fa.fa_pair_get_field(self.handle, None)[1]

    def field(self, layout=0):
        lvl, shp = fa.fa_pair_get_field(self.handle, None)
        shape = (3,) + shp if layout == 0 else shp + (3,)
        out = self._torch.empty(shape, dtype=self._torch.float32, device="cuda")
        fa.fa_pair_get_field(self.handle, out, layout)
        return out

    def warped(self):
        shp = self.level_shape()
        out = self._torch.empty(shp, dtype=self._torch.float32, device="cuda")
        fa.fa_pair_get_warped(self.handle, out)
        return out

    def progress(self):
        return fa.fa_pair_get_progress(self.handle)

    def set_state(self, d=None, m=None, v=None, t_done=0):
        fa.fa_pair_set_state(self.handle, d, m, v, t_done)

    def state(self):
        shp = self.level_shape()
        d, m, v = (self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda") for _ in range(3))
        fa.fa_pair_get_state(self.handle, d, m, v)
        return d, m, v

    def eval_gradient(self):
        shp = self.level_shape()
        g = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        loss = fa.fa_pair_eval_gradient(self.handle, g)
        return g, loss

    def direction(self):
        shp = self.level_shape()
        a = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        fa.fa_pair_get_direction(self.handle, a)
        return a

    def step_norm(self):
        return fa.fa_pair_get_step_norm(self.handle)

    def level_image(self, level, which):
        shp = fa.fa_pair_get_level_image(self.handle, level, which, None)
        out = self._torch.empty(shp, dtype=self._torch.float32, device="cuda")
        fa.fa_pair_get_level_image(self.handle, level, which, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            fa.fa_pair_destroy(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Inverse:
    """The post hoc inverse psi = phi^{-1} of a warp phi = id + d
    (fa_inverse.h): a (3, n0, n1, n2) float32 GPU tensor of displacements in
    voxels.

    >>> inv = Inverse(d, eta=0.1)
    >>> inv.set_schedule([4, 2, 1], [100, 50, 25]); inv.run()
    >>> e = inv.field()        # psi - id, (3, n0, n1, n2)
    """

    def __init__(self, d, *, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, beta1=0.9, beta2=0.999,
                 adam_eps=1e-8, stream=None):
        import torch
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = fa.fa_params_default()
        p.eta, p.sigma_grad, p.sigma_warp = eta, sigma_grad, sigma_warp
        p.adam_beta1, p.adam_beta2, p.adam_eps = beta1, beta2, adam_eps
        self.params = p
        self.shape = tuple(int(s) for s in d.shape[1:])
        self.handle = fa.fa_inverse_create(d, p, self.stream)
        self._keep = d   # alive until the stream has copied it
        self.total_iters = 0

    def set_schedule(self, scales, iters):
        fa.fa_inverse_set_schedule(self.handle, scales, iters)
        self.total_iters = int(sum(iters))

    def step(self, n):
        return fa.fa_inverse_step(self.handle, n)

    def run(self):
        return fa.fa_inverse_step(self.handle, 1 << 30)[0]

    def loss_history(self):
        return fa.fa_inverse_get_loss(self.handle, self.total_iters)

    def level_shape(self):
        return fa.fa_inverse_get_field(self.handle, None)[1]

    def field(self):
        shp = self.level_shape()
        out = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        fa.fa_inverse_get_field(self.handle, out)
        return out

    def eval_gradient(self):
        shp = self.level_shape()
        g = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        loss = fa.fa_inverse_eval_gradient(self.handle, g)
        return g, loss

    def set_splat(self, direct):
        fa.fa_inverse_set_splat(self.handle, direct)

    def close(self):
        if getattr(self, "handle", None):
            fa.fa_inverse_destroy(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Symmetric:
    """Symmetric registration (fa_symmetric.h): two half-way warps meet in the
    middle, then phi = phi_M o phi_F^{-1}.

    >>> s = Symmetric(fixed, moving, eta=0.5, window=5)
    >>> s.set_schedule([4, 2, 1], [200, 100, 50]); s.run()
    >>> d = s.finish([4, 2, 1], [100, 50, 25], eta=0.2)   # (3, n0, n1, n2)
    """

    def __init__(self, fixed, moving, *, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5,
                 cc_eps=1e-5, beta1=0.9, beta2=0.999, adam_eps=1e-8, use_jac=False, stream=None):
        import torch
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        p = fa.fa_params_default()
        p.eta, p.sigma_grad, p.sigma_warp, p.cc_window = eta, sigma_grad, sigma_warp, window
        p.cc_eps, p.adam_beta1, p.adam_beta2, p.adam_eps = cc_eps, beta1, beta2, adam_eps
        p.use_jac = 1 if use_jac else 0
        self.params = p
        self.shape = tuple(int(s) for s in fixed.shape)
        self.handle = fa.fa_sym_create(fixed, moving, p, self.stream)
        self._keep = (fixed, moving)
        self.total_iters = 0

    def set_schedule(self, scales, iters):
        fa.fa_sym_set_schedule(self.handle, scales, iters)
        self.total_iters = int(sum(iters))

    def step(self, n):
        return fa.fa_sym_step(self.handle, n)

    def run(self):
        return fa.fa_sym_step(self.handle, 1 << 30)[0]

    def loss_history(self):
        return fa.fa_sym_get_loss(self.handle, self.total_iters)

    def halfway(self):
        """(d_F, d_M) at the current level."""
        shp = fa.fa_sym_get_halfway(self.handle)[1]
        dF = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        dM = self._torch.empty((3,) + shp, dtype=self._torch.float32, device="cuda")
        fa.fa_sym_get_halfway(self.handle, dF, dM)
        return dF, dM

    def finish(self, scales, iters, *, eta=0.2, sigma_grad=1.0, sigma_warp=0.5, beta1=0.9, beta2=0.999,
               adam_eps=1e-8):
        """phi = phi_M o phi_F^{-1} (phi_F inverted over the given schedule):
        returns its displacement and stores the inverse fit's last cost in
        ``self.inverse_cost``."""
        p = fa.fa_params_default()
        p.eta, p.sigma_grad, p.sigma_warp = eta, sigma_grad, sigma_warp
        p.adam_beta1, p.adam_beta2, p.adam_eps = beta1, beta2, adam_eps
        d = self._torch.empty((3,) + self.shape, dtype=self._torch.float32, device="cuda")
        self.inverse_cost = fa.fa_sym_finish(self.handle, p, scales, iters, d)
        return d

    def close(self):
        if getattr(self, "handle", None):
            fa.fa_sym_destroy(self.handle)
            self.handle = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
