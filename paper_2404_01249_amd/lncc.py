"""The fused LNCC cost as a differentiable PyTorch loss.

:class:`LNCC` wraps one ``fa_lncc`` evaluator of the HIP library
(include/fa_lncc.h).  Calling it returns L = -mean_x cc(x) of the fixed image
and the moving image warped by the displacement d (voxel units, SoA
``(3, n0, n1, n2)``), with clipped w^3 windows (Section 4.4 cost; the
gradient is the Gateaux derivative of Section 4.4.2).  The backward pass
re-runs the fused kernel in gradient mode with the upstream derivative passed
as a device scalar, so nothing but the inputs is kept between forward and
backward and the window statistics are recomputed.  Gradients flow to ``d``
only; the images are treated as constants.
"""
from __future__ import annotations

import torch

from . import fa


class _LNCCFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, d, fixed, moving, ev):
        loss = torch.empty((), dtype=torch.float32, device=d.device)
        ev._eval(fixed, moving, d, loss=loss)
        ctx.save_for_backward(fixed, moving, d)
        ctx.ev = ev
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        fixed, moving, d = ctx.saved_tensors
        g = None
        if ctx.needs_input_grad[0]:
            scale = grad_loss.detach().to(torch.float32).reshape(()).contiguous()
            g = torch.empty_like(d)
            ctx.ev._eval(fixed, moving, d, grad=g, scale=scale)
        return g, None, None, None


class LNCC:
    """Fused LNCC loss for volumes of one shape.

    >>> lncc = LNCC((128, 128, 128), window=5)
    >>> loss = lncc(fixed, moving, d)       # d.requires_grad -> loss.backward() fills d.grad
    >>> loss, g = lncc.loss_and_grad(fixed, moving, d)   # one fused pass
    """

    def __init__(self, shape, window: int = 5, cc_eps: float = 1e-5, stream=None):
        self.shape = tuple(int(s) for s in shape)
        self.window = int(window)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = fa.fa_lncc_create(self.shape, self.window, cc_eps, self.stream)

    def _check(self, fixed, moving, d):
        if tuple(fixed.shape) != self.shape or tuple(moving.shape) != self.shape:
            raise ValueError(f"images must have shape {self.shape}")
        if tuple(d.shape) != (3,) + self.shape:
            raise ValueError(f"d must have shape {(3,) + self.shape}")
        if fixed.requires_grad or moving.requires_grad:
            raise ValueError("LNCC differentiates with respect to d only; detach the images")
        if torch.cuda.current_stream().cuda_stream != self.stream.cuda_stream:
            raise RuntimeError("LNCC must be called on the stream it was created with")

    def _eval(self, fixed, moving, d, loss=None, grad=None, scale=None):
        fa.fa_lncc_eval(self.handle, fixed, moving, d.detach(), loss, grad, scale)

    def __call__(self, fixed, moving, d):
        self._check(fixed, moving, d)
        return _LNCCFunction.apply(d, fixed, moving, self)

    def loss_and_grad(self, fixed, moving, d):
        """L and dL/dd from a single pass of the fused kernel."""
        self._check(fixed, moving, d)
        loss = torch.empty((), dtype=torch.float32, device=d.device)
        g = torch.empty((3,) + self.shape, dtype=torch.float32, device=d.device)
        self._eval(fixed, moving, d, loss=loss, grad=g)
        return loss, g

    def close(self):
        if getattr(self, "handle", None):
            fa.fa_lncc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
