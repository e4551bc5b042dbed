"""The stateless fused LNCC cost and gradient (include/fa_lncc.h) and its
PyTorch autograd wrapper, against the FP64 oracle.

Tolerances as for the registration step: loss |dL|/|L| <= 1e-5, gradient
||dg||_2/||g||_2 <= 1e-4.  The gradient is the Gateaux derivative of the
Section 4.4 cost with respect to the displacement (Section 4.4.2), which the
CPU suite pins to central differences of the oracle's loss.
"""
import numpy as np
import pytest

import bench_plain
import oracle as O
from paper_2404_01249_amd import LNCC, Pair, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_L = 1e-5
TOL_G = 1e-4


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def problem(shape, seed, max_norm=1.5):
    p = synth.blobs_pair(shape, seed=seed, n_blobs=12, sigma_range=(2.0, 5.0), field_sigma=3.0, field_max=2.0)
    d = synth.smooth_field(shape, seed + 1000, sigma=3.0, max_norm=max_norm)
    return p.fixed, p.moving, d


CASES = [((21, 37, 45), w) for w in (1, 3, 5, 7, 9)] + [((12, 131, 133), 5), ((12, 131, 133), 9), ((7, 5, 6), 9)]


@pytest.mark.parametrize("shape,window", CASES)
def test_loss_and_gradient_match_oracle(shape, window):
    print(f"lncc {shape} w={window}", flush=True)
    f, m, d = problem(shape, seed=21)
    g_ref, L_ref = O.gateaux_gradient(f.astype(np.float64), m.astype(np.float64), d.astype(np.float64), window, 1e-5)
    lncc = LNCC(shape, window=window)
    loss, g = lncc.loss_and_grad(dev(f), dev(m), dev(d))
    L, g = float(host(loss)), host(g)
    if window == 1:
        assert L == 0.0 and not g.any()          # a one-voxel window has no correlation
        return
    assert abs(L - L_ref) <= TOL_L * abs(L_ref), (L, L_ref)
    assert rel_l2(g, g_ref) <= TOL_G, rel_l2(g, g_ref)
    # the loss-only mode gives the same loss bit for bit
    loss2 = torch.empty((), dtype=torch.float32, device="cuda")
    lncc._eval(dev(f), dev(m), dev(d), loss=loss2)
    assert float(host(loss2)) == L
    lncc.close()


def test_same_as_registration_gradient():
    """At scale 1 the stateless call and the registration pair run the same
    kernel on the same data: identical results."""
    shape = (21, 37, 45)
    f, m, d = problem(shape, seed=22)
    lncc = LNCC(shape, window=5)
    loss, g = lncc.loss_and_grad(dev(f), dev(m), dev(d))
    pr = Pair(dev(f), dev(m), window=5)
    pr.set_schedule([1.0], [1])
    pr.set_state(dev(d), None, None, 0)
    g_pair, L_pair = pr.eval_gradient()
    assert np.array_equal(host(g), host(g_pair))
    assert float(host(loss)) == L_pair
    pr.close()
    lncc.close()


def test_autograd_backward_applies_upstream_derivative():
    shape = (21, 37, 45)
    f, m, d = problem(shape, seed=23)
    F, M = dev(f), dev(m)
    lncc = LNCC(shape, window=5)
    _, g = lncc.loss_and_grad(F, M, dev(d))
    dd = dev(d).requires_grad_(True)
    (3.0 * lncc(F, M, dd)).backward()
    assert np.array_equal(host(dd.grad), host(g * 3.0))
    # composed with other differentiable terms
    dd2 = dev(d).requires_grad_(True)
    total = lncc(F, M, dd2) + 0.1 * (dd2 * dd2).sum()
    total.backward()
    ref = host(g) + 0.2 * d.astype(np.float64)
    assert rel_l2(host(dd2.grad), ref) <= 1e-6
    # no graph: the loss-only pass
    with torch.no_grad():
        L = lncc(F, M, dev(d))
    assert not L.requires_grad
    lncc.close()


def test_rejects_bad_inputs():
    shape = (8, 9, 10)
    f, m, d = problem(shape, seed=24)
    lncc = LNCC(shape, window=3)
    with pytest.raises(ValueError):
        lncc(dev(f), dev(m), dev(d[:, :-1]))
    with pytest.raises(ValueError):
        lncc(dev(f).requires_grad_(True), dev(m), dev(d))
    lncc.close()


@pytest.mark.parametrize("window", [5, 9])
def test_blobs128_against_oracle_and_plain_autograd(window):
    """128^3 pair (blobs at twice the 64^3 sizes, field max 3 voxels), one
    evaluation at a smooth displacement of max norm 2 voxels."""
    print(f"lncc blobs128 w={window}", flush=True)
    p = synth.load("blobs128")
    d = synth.smooth_field(p.fixed.shape, 3, sigma=6.0, max_norm=2.0)
    F, M, D = dev(p.fixed), dev(p.moving), dev(d)
    lncc = LNCC(p.fixed.shape, window=window)
    loss, g = lncc.loss_and_grad(F, M, D)
    L, g = float(host(loss)), host(g)
    g_ref, L_ref = O.gateaux_gradient(p.fixed.astype(np.float64), p.moving.astype(np.float64),
                                      d.astype(np.float64), window, 1e-5)
    assert abs(L - L_ref) <= TOL_L * abs(L_ref), (L, L_ref)
    assert rel_l2(g, g_ref) <= TOL_G, rel_l2(g, g_ref)
    # the same loss written with stock PyTorch operators, differentiated by autograd (fp32)
    shape = p.fixed.shape
    ident = torch.stack(torch.meshgrid(*[torch.arange(n, device="cuda", dtype=torch.float32) for n in shape],
                                       indexing="ij"))[None]
    Dg = D[None].clone().requires_grad_(True)
    n = bench_plain.box(torch.ones((1, 1) + shape, device="cuda"), window)
    Lp = bench_plain.lncc_loss(F[None, None], bench_plain.warp(M[None, None], ident + Dg), window, 1e-5, n)
    gp, = torch.autograd.grad(Lp, Dg)
    print(f"plain autograd: loss rel {abs(float(Lp.detach()) - L_ref) / abs(L_ref):.2e}, "
          f"gradient rel {rel_l2(host(gp[0]), g_ref):.2e}", flush=True)
    assert abs(float(Lp.detach()) - L_ref) <= 1e-3 * abs(L_ref)
    assert rel_l2(host(gp[0]), g_ref) <= 2e-2
    lncc.close()


def fd_gradient_at(fixed, moving, d, y, c, window, eps, h):
    """FP64 central difference (h) of the oracle's cost in d_c(y).

    Moving d_c(y) changes the warped image J only at y, and the cost only
    through cc at the centres whose window holds y.  Those windows lie within
    2r of y, so the cost difference is the oracle's cc summed over those
    centres on a crop of y +- 2r (clipped at the volume's faces, so every
    window is the volume's own), divided by the volume's voxel count N."""
    r = window // 2
    n = fixed.shape
    lo = [max(0, y[a] - 2 * r) for a in range(3)]
    hi = [min(n[a], y[a] + 2 * r + 1) for a in range(3)]
    crop = tuple(slice(lo[a], hi[a]) for a in range(3))
    I = fixed[crop].astype(np.float64)
    pos = O.identity_grid(I.shape) + np.asarray(lo, np.float64)[:, None, None, None] + \
        d[(slice(None),) + crop].astype(np.float64)
    J = O.trilinear(moving, pos)
    yl = tuple(y[a] - lo[a] for a in range(3))
    cen = tuple(slice(max(0, y[a] - r) - lo[a], min(n[a], y[a] + r + 1) - lo[a]) for a in range(3))

    def cost_part(delta):
        p = pos[(slice(None),) + yl].copy()
        p[c] += delta
        Jp = J.copy()
        Jp[yl] = O.trilinear(moving, p.reshape(3, 1, 1, 1))[0, 0, 0]
        return -O.lncc_forward(I, Jp, window, eps)[0][cen].sum() / fixed.size

    return (cost_part(h) - cost_part(-h)) / (2.0 * h)


@pytest.mark.parametrize("window", [5, 9])
def test_blobs128_gradient_against_central_differences(window):
    """The fused gradient at 128^3 against FP64 central differences of the
    cost (h = 1e-3) at 64 seeded voxels, all three components.  Voxels whose
    sample x + d(x) lies within 2h of a cell boundary along any axis are
    redrawn: there the trilinear derivative jumps and a difference quotient
    does not measure it."""
    print(f"lncc blobs128 finite differences w={window}", flush=True)
    h = 1e-3
    p = synth.load("blobs128")
    d = synth.smooth_field(p.fixed.shape, 3, sigma=6.0, max_norm=2.0)
    lncc = LNCC(p.fixed.shape, window=window)
    _, g = lncc.loss_and_grad(dev(p.fixed), dev(p.moving), dev(d))
    g = host(g)
    lncc.close()
    moving = p.moving.astype(np.float64)
    rng = np.random.default_rng(128 + window)
    picked = []
    while len(picked) < 64:
        y = tuple(int(rng.integers(0, n)) for n in p.fixed.shape)
        frac = np.asarray([d[a][y] for a in range(3)], np.float64) % 1.0
        if np.all((frac > 2 * h) & (frac < 1 - 2 * h)):
            picked.append(y)
    got, ref = [], []
    for y in picked:
        for c in range(3):
            got.append(g[(c,) + y])
            ref.append(fd_gradient_at(p.fixed, moving, d, y, c, window, 1e-5, h))
    got, ref = np.asarray(got), np.asarray(ref)
    err = rel_l2(got, ref)
    print(f"finite differences w={window}: rel L2 {err:.2e}, max abs {np.abs(got - ref).max():.2e} "
          f"of max {np.abs(ref).max():.2e}", flush=True)
    assert err <= TOL_G
    assert np.abs(got - ref).max() <= TOL_G * np.abs(ref).max()
