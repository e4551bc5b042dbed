"""The path at the largest workload size: a 512^3 microscopy-like pair with an
LNCC window of 7^3 (the expansion-microscopy stand-in).

The full FP64 oracle does not fit in a test's time at 512^3, so it is run on
crops: the gradient at a voxel y depends only on the fixed image and the
warped moving image within 2r of y, and on the moving image around the
samples x + d(x) of those voxels.  A crop with that margin, clipped where it
meets the volume's faces (so the clipped windows are the volume's own),
reproduces the gradient at y, up to the factor N_crop / N of the mean in the
cost.  Sampled voxels include corners and faces.
"""
import numpy as np
import pytest

import oracle as O
from paper_2404_01249_amd import LNCC, Pair, evaluate, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE = (512, 512, 512)
WINDOW = 7
TOL_G = 1e-4


@pytest.fixture(scope="module")
def pair():
    print("generating the 512^3 pair", flush=True)
    return synth.microscopy_pair(SHAPE, seed=5)


def plane_waves(shape, seed, max_norm):
    """d_c(x) = sum of three seeded plane waves (float32): smooth, with
    gradients of order max_norm * 2 pi / 64 per voxel."""
    rng = np.random.default_rng(seed)
    ax = [np.arange(n, dtype=np.float32) for n in shape]
    d = np.zeros((3,) + shape, np.float32)
    for c in range(3):
        for _ in range(3):
            k = rng.uniform(-1.0, 1.0, 3) * (2 * np.pi / 64.0)
            ph = rng.uniform(0.0, 2 * np.pi)
            arg = (np.float32(k[0]) * ax[0])[:, None, None] + (np.float32(k[1]) * ax[1])[None, :, None] + \
                  (np.float32(k[2]) * ax[2])[None, None, :] + np.float32(ph)
            d[c] += np.sin(arg)
    d *= np.float32(max_norm / 3.0)
    return d


def oracle_gradient_at(fixed, moving, d, y, window, eps, dmax):
    """dU/dd at voxel y from the oracle on a crop around y (FP64)."""
    r = window // 2
    n = fixed.shape
    lo = [max(0, y[a] - 2 * r) for a in range(3)]
    hi = [min(n[a], y[a] + 2 * r + 1) for a in range(3)]
    crop = tuple(slice(lo[a], hi[a]) for a in range(3))
    I = fixed[crop].astype(np.float64)
    dc = d[(slice(None),) + crop].astype(np.float64)
    # the moving image around every sample x + d(x) of the crop
    m = int(np.ceil(dmax)) + 2
    mlo = [max(0, lo[a] - m) for a in range(3)]
    mhi = [min(n[a], hi[a] + m) for a in range(3)]
    mov = moving[mlo[0]:mhi[0], mlo[1]:mhi[1], mlo[2]:mhi[2]].astype(np.float64)
    pos = np.indices(I.shape, dtype=np.float64) + dc
    for a in range(3):
        pos[a] += lo[a] - mlo[a]
    J = O.trilinear(mov, pos)
    dLdJ, _ = O.lncc_grad_warped(I, J, window, eps)
    yc = tuple(y[a] - lo[a] for a in range(3))
    grad_p = O.trilinear_dpos(mov, pos[(slice(None),) + yc][:, None])[:, 0]
    return dLdJ[yc] * grad_p * (I.size / float(np.prod(n)))


def test_microscopy512_gradient_on_sampled_voxels(pair):
    print("512^3 gradient, window 7", flush=True)
    d = plane_waves(SHAPE, 51, 2.0)
    lncc = LNCC(SHAPE, window=WINDOW)
    loss, g = lncc.loss_and_grad(torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda(),
                                 torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    L = float(loss.cpu())
    assert -1.0 <= L <= 0.0 and np.isfinite(L)
    rng = np.random.default_rng(52)
    ys = [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(16)]
    ys += [(0, 0, 0), (511, 511, 511), (0, 255, 511), (511, 3, 200), (5, 511, 0), (256, 0, 300)]
    idx = torch.tensor([[y[0] for y in ys], [y[1] for y in ys], [y[2] for y in ys]], device="cuda")
    got = torch.stack([g[c][idx[0], idx[1], idx[2]] for c in range(3)], 1).cpu().numpy().astype(np.float64)
    dmax = float(np.abs(d).max()) * np.sqrt(3.0)
    ref = np.stack([oracle_gradient_at(pair.fixed, pair.moving, d, y, WINDOW, 1e-5, dmax) for y in ys])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"512^3 sampled gradient: rel l2 {err:.2e} over {len(ys)} voxels, loss {L:.6f}", flush=True)
    assert err <= TOL_G
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()
    lncc.close()


def test_microscopy512_short_registration(pair):
    """Scales 8, 4, 2, 1 at a few iterations each, at full size: the loss
    falls over the first level, nothing is non-finite and no voxel folds.
    (Within later levels the loss need not fall at first: the Adam moments
    carried across the transition and the fixed step length can raise it for
    a few iterations, as the oracle's own runs show.)"""
    print("512^3 short registration", flush=True)
    pr = Pair(torch.from_numpy(pair.fixed).cuda(), torch.from_numpy(pair.moving).cuda(), window=WINDOW)
    iters = [6, 4, 3, 2]
    pr.set_schedule([8.0, 4.0, 2.0, 1.0], iters)
    assert pr.run() == sum(iters)
    loss = pr.loss_history().astype(np.float64)
    assert np.all(np.isfinite(loss))
    assert loss[iters[0] - 1] < loss[0] - 0.01, loss[: iters[0]]
    d = pr.field()
    assert tuple(d.shape) == (3,) + SHAPE
    assert torch.isfinite(d).all()
    assert evaluate.singular_fraction(d) == 0.0
    pr.close()
