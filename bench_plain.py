"""Plain per-op PyTorch form of the same registration, for comparison only.

This is the algorithm the library runs (Algorithm 1 with the same readings:
clipped-window squared LNCC, Adam, Gaussian smoothing of the direction and of
the warp, eta / (2 max|s|) step scale, composition, corner-aligned trilinear
pyramid), written the way the paper's own implementation is described: with
stock PyTorch operators -- grid_sample for warps and the composition, conv3d
for window sums and Gaussians, autograd for the gradient, elementwise Adam.
It runs eagerly in float32 on the GPU.  It is a benchmark baseline, not a code
path of the library, and bench.py is its only user.
"""
import math

import torch
import torch.nn.functional as F


def _taps(sigma, device):
    s = float(torch.tensor(sigma, dtype=torch.float32))
    if not s > 0:
        return None
    R = int(math.ceil(3.0 * s))
    k = torch.arange(-R, R + 1, dtype=torch.float64)
    w = torch.exp(-(k * k) / (2 * s * s))
    return (w / w.sum()).to(device)


def smooth(x, sigma):
    """Separable Gaussian with replicate padding; x: (1, C, n0, n1, n2)."""
    w = _taps(sigma, x.device)
    if w is not None:
        w = w.to(x.dtype)
    if w is None:
        return x
    R = (w.numel() - 1) // 2
    C = x.shape[1]
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = w.numel()
        kern = w.view(1, 1, *shape).repeat(C, 1, 1, 1, 1)
        pad = [0, 0, 0, 0, 0, 0]
        pad[2 * (2 - ax)] = pad[2 * (2 - ax) + 1] = R
        x = F.conv3d(F.pad(x, pad, mode="replicate"), kern, groups=C)
    return x


def box(x, w):
    """Window sums over w^3 boxes clipped to the grid (zero padding)."""
    r = w // 2
    for ax in range(3):
        shape = [1, 1, 1]
        shape[ax] = w
        kern = torch.ones(x.shape[1], 1, *shape, device=x.device, dtype=x.dtype)
        pad = [0, 0, 0]
        pad[ax] = r
        x = F.conv3d(x, kern, padding=tuple(pad), groups=x.shape[1])
    return x


def lncc_loss(I, J, w, eps, n):
    stats = box(torch.cat([I, J, I * I, J * J, I * J], 1), w)
    SI, SJ, SII, SJJ, SIJ = stats.split(1, 1)
    cross = SIJ - SI * SJ / n
    vI = SII - SI * SI / n
    vJ = SJJ - SJ * SJ / n
    return -(cross * cross / (vI * vJ + eps)).mean()


def _grid(shape, p):
    """grid_sample grid (x, y, z order, align_corners=True) for voxel positions p (1,3,...)."""
    g = [2.0 * p[:, 2 - k] / (shape[2 - k] - 1) - 1.0 for k in range(3)]
    return torch.stack(g, -1)


def warp(img, p):
    return F.grid_sample(img, _grid(img.shape[2:], p), mode="bilinear", padding_mode="zeros",
                         align_corners=True)


def level_shape(shape, s):
    return tuple(max(1, int(math.floor(n / float(s) + 0.5))) for n in shape)


def register(fixed, moving, scales, iters, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5,
             cc_eps=1e-5, beta1=0.9, beta2=0.999, adam_eps=1e-8):
    shape = tuple(fixed.shape)
    If0, Im0 = fixed[None, None], moving[None, None]
    d = m = v = None
    t = 0
    losses = []
    for s, T in zip(scales, iters):
        ls = level_shape(shape, s)
        if float(s) == 1.0:
            If, Im = If0, Im0
        else:
            If = F.interpolate(smooth(If0, s / 2.0), size=ls, mode="trilinear", align_corners=True)
            Im = F.interpolate(smooth(Im0, s / 2.0), size=ls, mode="trilinear", align_corners=True)
        if d is None:
            d = torch.zeros((1, 3) + ls, device=fixed.device, dtype=fixed.dtype)
            m = torch.zeros_like(d)
            v = torch.zeros_like(d)
        else:
            cs = d.shape[2:]
            rho = torch.tensor([(ls[a] - 1) / (cs[a] - 1) for a in range(3)], device=d.device,
                               dtype=d.dtype).view(1, 3, 1, 1, 1)
            d = F.interpolate(d, size=ls, mode="trilinear", align_corners=True) * rho
            m = F.interpolate(m, size=ls, mode="trilinear", align_corners=True)
            v = F.interpolate(v, size=ls, mode="trilinear", align_corners=True)
        ident = torch.stack(torch.meshgrid(*[torch.arange(n, device=d.device, dtype=d.dtype) for n in ls],
                                           indexing="ij"))[None]
        n = box(torch.ones((1, 1) + ls, device=d.device, dtype=d.dtype), window)
        for _ in range(int(T)):
            t += 1
            dd = d.detach().requires_grad_(True)
            loss = lncc_loss(If, warp(Im, ident + dd), window, cc_eps, n)
            g, = torch.autograd.grad(loss, dd)
            losses.append(loss.detach())
            with torch.no_grad():
                m = beta1 * m + (1 - beta1) * g
                v = beta2 * v + (1 - beta2) * g * g
                a = (m / (1 - beta1 ** t)) / ((v / (1 - beta2 ** t)).sqrt() + adam_eps)
                sm = smooth(a, sigma_grad)
                M = sm.norm(dim=1).amax()
                u = torch.where(M > 0, -eta / (2 * M), torch.zeros_like(M)) * sm
                d = u + torch.cat([warp(d[:, c:c + 1], ident + u) for c in range(3)], 1)
                d = smooth(d, sigma_warp)
    return d[0], torch.stack(losses).cpu().numpy() if losses else []


if __name__ == "__main__":
    # Standalone run for kernel traces and counters of the plain form:
    #   python3 bench_plain.py --workload tissue160 --scales 1 --iters 3
    import argparse
    import os
    import sys
    import time

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_2404_01249_amd import synth

    ap = argparse.ArgumentParser(description="plain per-op PyTorch registration (comparison baseline)")
    ap.add_argument("--workload", default="tissue160")
    ap.add_argument("--scales", type=float, nargs="+", default=None)
    ap.add_argument("--iters", type=int, nargs="+", default=None)
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--calib", action="store_true",
                    help="first run a 256 MiB read + 256 MiB write elementwise kernel "
                         "(reference for hardware byte counters)")
    args = ap.parse_args()
    if args.calib:
        x = torch.ones(64 * 1024 * 1024, device="cuda")
        y = torch.empty_like(x)
        torch.add(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    p = synth.load(args.workload)
    scales = args.scales or p.scales
    iters = args.iters or p.iters
    fixed = torch.from_numpy(p.fixed).cuda()
    moving = torch.from_numpy(p.moving).cuda()
    for r in range(args.reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d, losses = register(fixed, moving, scales, iters, window=p.window)
        torch.cuda.synchronize()
        print(f"plain registration {r}: scales {scales} iters {iters}: {time.perf_counter() - t0:.3f} s, "
              f"final loss {float(losses[-1]):.6f}", flush=True)
