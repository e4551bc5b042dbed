"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks one oracle function against something other than itself:
a special case with a known exact answer, an invariant the paper states, a
library routine that implements the same definition (SciPy, NumPy, PyTorch
CPU in float64), brute force on tiny inputs, or central finite differences.
The cases are chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch
import torch.nn.functional as F

import oracle as O

RNG = np.random.default_rng(1234)


def rand(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


# ---------------------------------------------------------------------------
# Trilinear warp
# ---------------------------------------------------------------------------

def test_identity_warp_reproduces_image_bitwise():
    I = rand(5, 6, 7, seed=1)
    J = O.warp_image(I, np.zeros((3, 5, 6, 7)))
    assert np.array_equal(J, I)


@pytest.mark.parametrize("shift", [(1, 0, 0), (0, -2, 0), (0, 0, 3), (1, -1, 2)])
def test_integer_shift_is_exact_with_zero_fill(shift):
    I = rand(5, 6, 7, seed=2)
    d = np.zeros((3, 5, 6, 7))
    for a in range(3):
        d[a] = shift[a]
    J = O.warp_image(I, d)
    ref = np.zeros_like(I)
    src = tuple(slice(max(0, s), n + min(0, s)) for s, n in zip(shift, I.shape))
    dst = tuple(slice(max(0, -s), n + min(0, -s)) for s, n in zip(shift, I.shape))
    ref[dst] = I[src]
    assert np.array_equal(J, ref)


def test_linear_image_reproduced_inside_domain():
    n = (6, 7, 8)
    x = np.indices(n, dtype=np.float64)
    a = np.array([0.3, -1.2, 0.7])
    I = 2.0 + sum(a[k] * x[k] for k in range(3))
    p = RNG.uniform(0.0, 1.0, size=(3, 200)) * (np.array(n)[:, None] - 1.0001)
    T = O.trilinear(I, p)
    np.testing.assert_allclose(T, 2.0 + (a[:, None] * p).sum(0), rtol=0, atol=1e-12)
    G = O.trilinear_dpos(I, p)
    np.testing.assert_allclose(G, np.broadcast_to(a[:, None], G.shape), rtol=0, atol=1e-12)


def test_trilinear_matches_scipy_grid_constant():
    """scipy order-1 spline with 'grid-constant' padding is trilinear
    interpolation with zero values beyond the grid, corner by corner."""
    I = rand(5, 6, 7, seed=3)
    p = RNG.uniform(-1.5, 1.0, size=(3, 500)) * 1.0 + np.array([2.0, 2.5, 3.0])[:, None] * RNG.uniform(0, 2, size=(3, 500))
    ref = ndi.map_coordinates(I, p, order=1, mode="grid-constant", cval=0.0)
    np.testing.assert_allclose(O.trilinear(I, p), ref, rtol=0, atol=1e-12)


def test_trilinear_matches_torch_grid_sample_align_corners_zeros():
    n = (5, 6, 7)
    I = rand(*n, seed=4)
    d = 1.5 * rand(3, *n, seed=5)
    J = O.warp_image(I, d)
    p = np.indices(n, dtype=np.float64) + d
    # grid_sample wants (x, y, z) = (axis2, axis1, axis0) normalised to [-1, 1]
    g = np.stack([2.0 * p[2 - k] / (n[2 - k] - 1) - 1.0 for k in range(3)], -1)
    ref = F.grid_sample(torch.from_numpy(I)[None, None], torch.from_numpy(g)[None],
                        mode="bilinear", padding_mode="zeros", align_corners=True)
    np.testing.assert_allclose(J, ref[0, 0].numpy(), rtol=0, atol=1e-12)


def test_position_derivative_central_differences_inside_cell():
    """T is linear along each axis inside a cell, so a central difference that
    stays in the cell equals the derivative up to rounding."""
    I = rand(6, 6, 6, seed=6)
    q = RNG.integers(0, 4, size=(3, 100)).astype(np.float64)
    p = q + RNG.uniform(0.1, 0.9, size=(3, 100))
    G = O.trilinear_dpos(I, p)
    h = 0.05
    for a in range(3):
        e = np.zeros((3, 1))
        e[a] = h
        fd = (O.trilinear(I, p + e) - O.trilinear(I, p - e)) / (2 * h)
        np.testing.assert_allclose(G[a], fd, rtol=0, atol=1e-11)


def test_position_derivative_is_right_derivative_at_integer():
    I = rand(5, 5, 5, seed=7)
    p = np.array([[2.0], [1.0], [3.0]])
    G = O.trilinear_dpos(I, p)
    # right derivative along axis 0 at an integer point: I[3,1,3] - I[2,1,3]
    assert G[0, 0] == pytest.approx(I[3, 1, 3] - I[2, 1, 3], abs=1e-14)
    assert G[2, 0] == pytest.approx(I[2, 1, 4] - I[2, 1, 3], abs=1e-14)


# ---------------------------------------------------------------------------
# Box sums and LNCC
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,r", [((5, 6, 7), 1), ((5, 6, 7), 2), ((3, 9, 4), 2), ((2, 3, 11), 3)])
def test_box_sum_brute_force(shape, r):
    f = rand(*shape, seed=8)
    S = O.box_sum(f, r)
    ref = np.zeros_like(f)
    for i in np.ndindex(*shape):
        lo = [max(0, i[a] - r) for a in range(3)]
        hi = [min(shape[a], i[a] + r + 1) for a in range(3)]
        ref[i] = f[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].sum()
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-12)
    w = 2 * r + 1
    uf = ndi.uniform_filter(f, size=w, mode="constant", cval=0.0) * w ** 3
    np.testing.assert_allclose(S, uf, rtol=0, atol=1e-11)
    cnt = O.window_count(shape, r)
    assert cnt[tuple(min(r, n - 1 - r) if n > 2 * r else 0 for n in shape)] <= w ** 3


@pytest.mark.parametrize("shape,w", [((5, 6, 7), 3), ((6, 5, 7), 5), ((4, 7, 3), 5)])
def test_lncc_equals_windowed_squared_pearson(shape, w):
    """At eps = 0, cc(x) is the squared Pearson correlation of I and J over the
    clipped window (np.corrcoef, an independent routine)."""
    I = rand(*shape, seed=9)
    J = 0.5 * I + rand(*shape, seed=10)
    cc, L, _ = O.lncc_forward(I, J, w, 0.0)
    r = w // 2
    ref = np.zeros(shape)
    for i in np.ndindex(*shape):
        sl = tuple(slice(max(0, i[a] - r), min(shape[a], i[a] + r + 1)) for a in range(3))
        ref[i] = np.corrcoef(I[sl].ravel(), J[sl].ravel())[0, 1] ** 2
    np.testing.assert_allclose(cc, ref, rtol=1e-10, atol=1e-12)
    assert L == pytest.approx(-ref.mean(), rel=1e-12)


def test_lncc_self_is_maximal_and_affine_invariant():
    I = rand(6, 7, 8, seed=11)
    cc_self, L_self, _ = O.lncc_forward(I, I, 5, 0.0)
    np.testing.assert_allclose(cc_self, 1.0, rtol=0, atol=1e-12)
    for a, b in [(2.5, 0.3), (-0.7, 4.0), (1e-2, -1.0)]:
        cc_aff, _, _ = O.lncc_forward(I, a * I + b, 5, 0.0)
        np.testing.assert_allclose(cc_aff, 1.0, rtol=0, atol=1e-9)
    J = rand(6, 7, 8, seed=12)
    cc, L, _ = O.lncc_forward(I, J, 5, 0.0)
    assert np.all(cc >= -1e-15) and np.all(cc <= 1 + 1e-12)
    assert L > L_self
    cc2, _, _ = O.lncc_forward(J, I, 5, 0.0)
    np.testing.assert_allclose(cc, cc2, rtol=1e-12, atol=1e-14)
    cc3, _, _ = O.lncc_forward(3.0 * I - 1.0, 0.5 * J + 2.0, 5, 0.0)
    np.testing.assert_allclose(cc3, cc, rtol=1e-8, atol=1e-12)


def test_lncc_eps_regularises_flat_windows():
    I = np.ones((5, 5, 5))
    cc, L, _ = O.lncc_forward(I, I, 3, 1e-5)
    assert np.all(cc == 0.0) and L == 0.0
    cc0, L0, _ = O.lncc_forward(I, I, 3, 0.0)      # D == 0 everywhere -> defined as 0
    assert np.all(cc0 == 0.0)


def test_lncc_grad_central_differences():
    I = rand(5, 6, 7, seed=13)
    J = 0.3 * I + rand(5, 6, 7, seed=14)
    dJ, L = O.lncc_grad_warped(I, J, 3, 1e-3)
    h = 1e-6
    for idx in [(0, 0, 0), (2, 3, 4), (4, 5, 6), (1, 0, 6), (3, 2, 1)]:
        Jp, Jm = J.copy(), J.copy()
        Jp[idx] += h
        Jm[idx] -= h
        fd = (O.lncc_forward(I, Jp, 3, 1e-3)[1] - O.lncc_forward(I, Jm, 3, 1e-3)[1]) / (2 * h)
        assert dJ[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def _torch_lncc_loss(I, J, w, eps):
    """Independent float64 PyTorch LNCC: box sums by conv3d with a ones kernel
    on a zero-padded volume, counts by the same conv of ones."""
    k = torch.ones(1, 1, w, w, w, dtype=torch.float64)
    r = w // 2

    def box(x):
        return F.conv3d(x[None, None], k, padding=r)[0, 0]
    n = box(torch.ones_like(I))
    SI, SJ, SII, SJJ, SIJ = box(I), box(J), box(I * I), box(J * J), box(I * J)
    cross = SIJ - SI * SJ / n
    vI = SII - SI * SI / n
    vJ = SJJ - SJ * SJ / n
    return -(cross * cross / (vI * vJ + eps)).mean()


@pytest.mark.parametrize("w", [3, 5])
def test_lncc_grad_matches_torch_autograd(w):
    I = rand(6, 7, 5, seed=15)
    J = 0.5 * I + 0.5 * rand(6, 7, 5, seed=16)
    dJ, L = O.lncc_grad_warped(I, J, w, 1e-5)
    It = torch.from_numpy(I)
    Jt = torch.from_numpy(J).requires_grad_(True)
    Lt = _torch_lncc_loss(It, Jt, w, 1e-5)
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    np.testing.assert_allclose(dJ, Jt.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_gateaux_gradient_central_differences():
    n = (7, 8, 9)
    x = np.indices(n, dtype=np.float64)
    fixed = np.sin(0.7 * x[0]) * np.cos(0.5 * x[1]) + 0.3 * np.sin(0.9 * x[2]) + 0.05 * rand(*n, seed=17)
    moving = np.sin(0.7 * x[0] + 0.3) * np.cos(0.5 * x[1] - 0.2) + 0.3 * np.sin(0.9 * x[2] + 0.1)
    d = 0.6 * rand(3, *n, seed=18)
    g, L = O.gateaux_gradient(fixed, moving, d, 3, 1e-5)
    h = 1e-3
    rng = np.random.default_rng(19)
    checked = 0
    while checked < 24:
        idx = tuple(int(rng.integers(0, s)) for s in n)
        c = int(rng.integers(0, 3))
        pos = idx[c] + d[(c,) + idx]
        if abs(pos - round(pos)) < 2 * h:
            continue
        dp, dm = d.copy(), d.copy()
        dp[(c,) + idx] += h
        dm[(c,) + idx] -= h
        Lp = O.lncc_forward(fixed, O.warp_image(moving, dp), 3, 1e-5)[1]
        Lm = O.lncc_forward(fixed, O.warp_image(moving, dm), 3, 1e-5)[1]
        fd = (Lp - Lm) / (2 * h)
        assert g[(c,) + idx] == pytest.approx(fd, rel=2e-5, abs=1e-9)
        checked += 1


def test_gateaux_gradient_matches_torch_grid_sample_autograd():
    n = (6, 7, 8)
    fixed = rand(*n, seed=20)
    moving = ndi.gaussian_filter(rand(*n, seed=21), 1.0)
    d = 0.8 * rand(3, *n, seed=22)
    g, L = O.gateaux_gradient(fixed, moving, d, 3, 1e-5)
    dt = torch.from_numpy(d).requires_grad_(True)
    p = torch.from_numpy(np.indices(n, dtype=np.float64)) + dt
    grid = torch.stack([2.0 * p[2 - k] / (n[2 - k] - 1) - 1.0 for k in range(3)], -1)
    J = F.grid_sample(torch.from_numpy(moving)[None, None], grid[None], mode="bilinear",
                      padding_mode="zeros", align_corners=True)[0, 0]
    Lt = _torch_lncc_loss(torch.from_numpy(fixed), J, 3, 1e-5)
    Lt.backward()
    assert L == pytest.approx(Lt.item(), rel=1e-12)
    # away from integer sample coordinates the two derivatives coincide
    frac = np.abs((np.indices(n) + d) - np.round(np.indices(n) + d))
    mask = frac > 1e-6
    np.testing.assert_allclose(g[mask], dt.grad.numpy()[mask], rtol=1e-8, atol=1e-14)


# ---------------------------------------------------------------------------
# Eulerian direction (use_jac)
# ---------------------------------------------------------------------------

def test_eulerian_direction_is_identity_at_the_identity_map():
    g = rand(3, 5, 6, 7, seed=40)
    assert np.array_equal(O.eulerian_direction(g, np.zeros_like(g)), g)


def _affine_field(n, A, b):
    x = np.indices(n, dtype=np.float64)
    return np.einsum("ca,a...->c...", A, x) + np.asarray(b)[:, None, None, None]


def test_eulerian_direction_of_an_affine_map_is_the_transposed_jacobian():
    """d = A x + b: J(phi) = I + A everywhere (central and one-sided differences
    are exact for a linear field), and the direction is (I + A)^T g.  A is not
    symmetric, so a transposed Jacobian fails."""
    n = (5, 6, 7)
    A = np.array([[0.1, -0.3, 0.2], [0.05, 0.2, -0.15], [0.4, 0.0, -0.1]])
    d = _affine_field(n, A, [0.3, -0.2, 0.1])
    g = rand(3, *n, seed=41)
    ref = np.einsum("ca,c...->a...", np.eye(3) + A, g)
    np.testing.assert_allclose(O.eulerian_direction(g, d), ref, rtol=1e-12, atol=1e-13)


def test_eulerian_direction_predicts_the_cost_along_the_composed_path():
    """Definition of the Eulerian differential (Section 4.4.2): the derivative
    of U(phi o (id + eps v)) at eps = 0 is <J(phi)^T dU/dphi, v>.  With an
    affine d, phi o (id + eps v) = phi + eps (I + A) v exactly (trilinear
    interpolation reproduces an affine field), so central differences of the
    cost along the composed path pin the direction; v vanishes on the faces so
    that no sample leaves the grid.  The Gateaux direction alone misses the
    term and fails the same check."""
    n = (10, 11, 12)
    fixed = ndi.gaussian_filter(rand(*n, seed=42), 1.5)
    moving = ndi.gaussian_filter(rand(*n, seed=43), 1.5)
    A = np.array([[0.15, -0.2, 0.1], [0.1, -0.12, 0.2], [-0.25, 0.05, 0.1]])
    d = _affine_field(n, A, [0.37, -0.41, 0.23])
    v = np.stack([ndi.gaussian_filter(rand(*n, seed=44 + c), 1.0) for c in range(3)])
    v[:, [0, -1], :, :] = 0.0
    v[:, :, [0, -1], :] = 0.0
    v[:, :, :, [0, -1]] = 0.0
    g, _ = O.gateaux_gradient(fixed, moving, d, 3, 1e-5)
    eps = 1e-5
    Up = O.lncc_forward(fixed, O.warp_image(moving, O.compose(d, eps * v)), 3, 1e-5)[1]
    Um = O.lncc_forward(fixed, O.warp_image(moving, O.compose(d, -eps * v)), 3, 1e-5)[1]
    fd = (Up - Um) / (2 * eps)
    euler = float((O.eulerian_direction(g, d) * v).sum())
    gateaux = float((g * v).sum())
    assert euler == pytest.approx(fd, rel=1e-4)
    assert abs(gateaux - fd) > 0.05 * abs(fd)


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------

def test_adam_closed_forms():
    g = rand(3, 4, 5, 6, seed=23) * 1e-3
    a, m, v = O.adam_update(g, np.zeros_like(g), np.zeros_like(g), 1, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(a, g / (np.abs(g) + 1e-8), rtol=1e-12)
    m = v = np.zeros_like(g)
    for t in range(1, 30):
        a, m, v = O.adam_update(g, m, v, t, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(a, g / (np.abs(g) + 1e-8), rtol=1e-9)


def test_adam_matches_torch_optim_adam():
    """torch.optim.Adam with lr = 1 moves a parameter by exactly -a."""
    rng = np.random.default_rng(24)
    p = torch.zeros(2, 3, 4, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1.0, betas=(0.9, 0.999), eps=1e-8)
    m = v = np.zeros((2, 3, 4))
    for t in range(1, 12):
        g = rng.standard_normal((2, 3, 4)) * 10.0 ** rng.uniform(-7, -3)
        a, m, v = O.adam_update(g, m, v, t, 0.9, 0.999, 1e-8)
        before = p.detach().clone()
        p.grad = torch.from_numpy(g)
        opt.step()
        np.testing.assert_allclose((before - p.detach()).numpy(), a, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# Gaussian smoothing
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.4, 0.5, 1.0, 2.0, 6.0])
def test_gaussian_weights(sigma):
    w = O.gaussian_weights(sigma)
    R = math.ceil(3 * float(np.float32(sigma)))
    assert len(w) == 2 * R + 1
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_array_equal(w, w[::-1])
    assert np.argmax(w) == R


@pytest.mark.parametrize("sigma", [0.4, 0.5, 1.0, 2.0, 6.0])
def test_gaussian_tap_values_match_independent_sampled_gaussians(sigma):
    """Tap values against two independent samplings of the same kernel:
    the impulse response of scipy.ndimage.gaussian_filter1d (truncate chosen
    so its radius int(truncate sigma + 1/2) is ceil(3 sigma)) and
    scipy.signal.windows.gaussian normalised to sum 1.  A sigma-for-sigma^2
    slip (equal at sigma = 1 only) or a wrong radius fails here."""
    from scipy.signal import windows
    s = float(np.float32(sigma))     # the library receives sigma as float32
    R = math.ceil(3 * s)
    w = O.gaussian_weights(sigma)
    impulse = np.zeros(4 * R + 3)
    impulse[2 * R + 1] = 1.0
    resp = ndi.gaussian_filter1d(impulse, s, mode="constant", truncate=R / s)
    ref1 = resp[R + 1: 3 * R + 2]
    assert np.count_nonzero(resp) == 2 * R + 1
    np.testing.assert_allclose(w, ref1, rtol=1e-13, atol=0)
    g = windows.gaussian(2 * R + 1, std=s, sym=True)
    np.testing.assert_allclose(w, g / g.sum(), rtol=1e-13, atol=0)
    # the ratio of neighbouring taps is exp(-(2k+1) / (2 sigma^2)), computed here
    # from the definition rather than from the oracle's own expression
    k = np.arange(0, R)
    np.testing.assert_allclose(w[R + k + 1] / w[R + k], np.exp(-(2 * k + 1) / (2 * s * s)), rtol=1e-12)


@pytest.mark.parametrize("sigma", [0.5, 1.0, 2.0])
def test_gaussian_matches_scipy_correlate_nearest(sigma):
    """scipy.ndimage.correlate1d with mode='nearest' is replicate padding."""
    f = rand(3, 9, 8, 7, seed=25)
    w = O.gaussian_weights(sigma)
    ref = f.copy()
    for ax in (1, 2, 3):
        ref = ndi.correlate1d(ref, w, axis=ax, mode="nearest")
    np.testing.assert_allclose(O.gaussian_smooth(f, sigma), ref, rtol=0, atol=1e-13)


def test_gaussian_preserves_constants_and_interior_linear():
    c = np.full((3, 8, 9, 10), 0.37)
    np.testing.assert_allclose(O.gaussian_smooth(c, 1.0), c, rtol=0, atol=1e-15)
    x = np.indices((12, 12, 12), dtype=np.float64)
    lin = 0.2 * x[0] - 0.5 * x[1] + 0.1 * x[2] + 3.0
    out = O.gaussian_smooth(lin[None], 1.0)[0]
    R = 3
    inner = (slice(R, -R),) * 3
    np.testing.assert_allclose(out[inner], lin[inner], rtol=0, atol=1e-12)


def test_gaussian_separable_equals_direct_3d_and_numpy_convolve():
    f = rand(1, 6, 5, 7, seed=26)
    s = 0.8
    w = O.gaussian_weights(s)
    R = len(w) // 2
    ref = np.zeros_like(f[0])
    n = f.shape[1:]
    for i in np.ndindex(*n):
        acc = 0.0
        for a in range(-R, R + 1):
            for b in range(-R, R + 1):
                for c in range(-R, R + 1):
                    j = (min(max(i[0] + a, 0), n[0] - 1), min(max(i[1] + b, 0), n[1] - 1),
                         min(max(i[2] + c, 0), n[2] - 1))
                    acc += w[a + R] * w[b + R] * w[c + R] * f[(0,) + j]
        ref[i] = acc
    np.testing.assert_allclose(O.gaussian_smooth(f, s)[0], ref, rtol=0, atol=1e-13)
    # 1-D special case against numpy.convolve on an edge-padded line
    line = rand(20, seed=27)
    padded = np.pad(line, R, mode="edge")
    ref1 = np.convolve(padded, w[::-1], mode="valid")
    vol = np.broadcast_to(line, (1, 1, 1, 20)).copy()
    np.testing.assert_allclose(O.gaussian_smooth(vol, s)[0, 0, 0], ref1, rtol=0, atol=1e-14)


def test_gaussian_nonpositive_sigma_is_identity():
    f = rand(3, 4, 5, 6, seed=28)
    assert np.array_equal(O.gaussian_smooth(f, 0.0), f)
    assert np.array_equal(O.gaussian_smooth(f, -1.0), f)


# ---------------------------------------------------------------------------
# Step normalisation (Appendix E) and composition
# ---------------------------------------------------------------------------

def test_normalised_step_has_max_norm_eta_over_two():
    s = rand(3, 6, 7, 8, seed=29)
    for eta in (0.25, 0.5, 2.0):
        u, M = O.normalise_step(s, eta)
        assert np.sqrt((u * u).sum(0)).max() == pytest.approx(eta / 2, rel=1e-14)
        assert np.all(np.sign(u) == -np.sign(s))
    u, M = O.normalise_step(np.zeros((3, 2, 2, 2)), 0.5)
    assert M == 0 and np.all(u == 0)


def test_normalised_smooth_step_is_a_diffeomorphism():
    """Appendix E's theorem: with the scale eta / (2 sup|v|) and eta < 1 the
    update id + u has a positive Jacobian determinant everywhere."""
    a = rand(3, 16, 16, 16, seed=30)
    a = a / (np.abs(a) + 1e-8)              # Adam-normalised direction, |a_c| ~ 1
    s = O.gaussian_smooth(a, 1.0)
    u, _ = O.normalise_step(s, 0.5)
    assert O.jacobian_det(u).min() > 0


def test_compose_special_cases():
    n = (6, 7, 8)
    d = rand(3, *n, seed=31)
    zero = np.zeros((3,) + n)
    assert np.array_equal(O.compose(d, zero), d)                     # phi o id = phi
    u = 0.4 * rand(3, *n, seed=32)
    np.testing.assert_array_equal(O.compose(zero, u), u)             # id o (id+u) = id+u
    c = np.stack([np.full(n, 0.3), np.full(n, -0.2), np.full(n, 0.1)])
    b = np.stack([np.full(n, 0.25), np.full(n, 0.5), np.full(n, -0.4)])
    out = O.compose(c, b)
    inner = (slice(None), slice(0, n[0] - 1), slice(0, n[1] - 1), slice(1, n[2]))
    np.testing.assert_allclose(out[inner], (b + c)[inner], rtol=0, atol=1e-14)
    # an integer translation shifts d exactly (zero fill at the far edge)
    ui = np.zeros((3,) + n)
    ui[1] = 1.0
    out = O.compose(d, ui)
    np.testing.assert_array_equal(out[:, :, :-1, :], d[:, :, 1:, :] + ui[:, :, :-1, :])
    np.testing.assert_array_equal(out[:, :, -1, :], ui[:, :, -1, :])


def test_compose_of_affine_maps_is_their_composition():
    """(id + A x + b) o (id + u) for linear d = A x + b and constant u stays
    inside the grid: d'(x) = u + A (x + u) + b, exactly."""
    n = (8, 8, 8)
    x = np.indices(n, dtype=np.float64)
    A = np.array([[0.05, -0.02, 0.01], [0.03, 0.04, -0.05], [-0.01, 0.02, 0.03]])
    b = np.array([0.2, -0.1, 0.3])
    d = np.einsum("ij,j...->i...", A, x) + b[:, None, None, None]
    u = np.broadcast_to(np.array([0.3, -0.45, 0.2])[:, None, None, None], (3,) + n).copy()
    out = O.compose(d, u)
    ref = u + np.einsum("ij,j...->i...", A, x + u) + b[:, None, None, None]
    inner = (slice(None), slice(0, 7), slice(1, 8), slice(0, 7))
    np.testing.assert_allclose(out[inner], ref[inner], rtol=0, atol=1e-13)


# ---------------------------------------------------------------------------
# Pyramid and level transitions
# ---------------------------------------------------------------------------

def test_level_shapes():
    assert O.level_shape((160, 192, 224), 4) == (40, 48, 56)
    assert O.level_shape((160, 192, 224), 2) == (80, 96, 112)
    assert O.level_shape((64, 64, 64), 1) == (64, 64, 64)
    assert O.level_shape((5, 7, 9), 2) == (3, 4, 5)
    assert O.level_shape((3, 3, 3), 8) == (1, 1, 1)


def test_downsample_is_blur_then_corner_aligned_resample():
    """Blur pinned by the Gaussian tests; the resample against scipy.ndimage.zoom
    (order 1, grid_mode=False = corner-aligned trilinear)."""
    I = rand(16, 12, 20, seed=33)
    out = O.downsample_image(I, 2.0)
    assert out.shape == (8, 6, 10)
    blurred = O.gaussian_smooth(I[None], 1.0)[0]
    ref = ndi.zoom(blurred, (8 / 16, 6 / 12, 10 / 20), order=1, mode="nearest", grid_mode=False)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)
    c = np.full((16, 12, 20), 0.7)
    np.testing.assert_allclose(O.downsample_image(c, 4.0), 0.7, rtol=0, atol=1e-14)
    assert np.array_equal(O.downsample_image(I, 1.0), I)


def test_upsample_state_linear_field_with_rescale():
    nc, nf = (5, 6, 7), (9, 11, 13)
    xc = np.indices(nc, dtype=np.float64)
    A = np.array([[0.1, 0.0, -0.05], [0.02, -0.1, 0.0], [0.0, 0.03, 0.07]])
    d = np.einsum("ij,j...->i...", A, xc)
    m = np.stack([np.full(nc, 1.5), np.full(nc, -2.0), np.full(nc, 0.25)])
    d2, m2, v2 = O.upsample_state(d, m, np.abs(m), nf)
    xf = np.indices(nf, dtype=np.float64)
    sc = np.array([(nc[a] - 1) / (nf[a] - 1) for a in range(3)])
    rho = 1.0 / sc
    # the coarse field evaluated at coarse positions, expressed in fine voxels
    ref = np.einsum("ij,j...->i...", A, xf * sc[:, None, None, None]) * rho[:, None, None, None]
    np.testing.assert_allclose(d2, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(m2, np.broadcast_to(m[:, :1, :1, :1], m2.shape), rtol=0, atol=1e-14)
    np.testing.assert_allclose(v2, np.abs(m2), rtol=0, atol=1e-14)


def test_trilinear_upsampling_keeps_a_diffeomorphism():
    """Section 4.5: trilinear upsampling of a diffeomorphic field does not
    overshoot and keeps det J > 0."""
    nc = (10, 10, 10)
    x = np.indices(nc, dtype=np.float64)
    d = np.stack([1.2 * np.sin(0.5 * x[1]) * np.cos(0.3 * x[2]),
                  0.8 * np.sin(0.4 * x[0]),
                  1.0 * np.cos(0.35 * x[0] + 0.2 * x[1])])
    assert O.jacobian_det(d).min() > 0
    d2, _, _ = O.upsample_state(d, d, d, (19, 19, 19))
    assert O.jacobian_det(d2).min() > 0


# ---------------------------------------------------------------------------
# Evaluation helpers
# ---------------------------------------------------------------------------

def test_jacobian_det_and_singular_fraction():
    n = (6, 6, 6)
    assert np.allclose(O.jacobian_det(np.zeros((3,) + n)), 1.0)
    x = np.indices(n, dtype=np.float64)
    A = np.array([[0.1, 0.2, 0.0], [-0.1, 0.3, 0.05], [0.0, 0.1, -0.2]])
    d = np.einsum("ij,j...->i...", A, x)
    np.testing.assert_allclose(O.jacobian_det(d), np.linalg.det(np.eye(3) + A), rtol=1e-12)
    fold = np.zeros((3,) + n)
    fold[0] = -2.0 * x[0]
    assert O.singular_fraction(fold) == 1.0


def test_dice_and_nearest_label_warp():
    lab = np.random.default_rng(34).integers(0, 4, size=(6, 7, 8))
    assert O.dice(lab, lab, range(4)) == 1.0
    assert O.dice(lab, (lab + 1) % 4, range(4)) == 0.0
    half = np.where(lab == 0, 1, lab)            # class 0 vanishes, class 1 grows
    n0, n1 = (lab == 0).sum(), (lab == 1).sum()
    assert O.dice(lab, half, [1]) == pytest.approx(2 * n1 / (n1 + n1 + n0))
    assert np.array_equal(O.warp_labels_nearest(lab, np.zeros((3, 6, 7, 8))), lab)
    d = np.zeros((3, 6, 7, 8))
    d[2] = 1.0
    w = O.warp_labels_nearest(lab, d)
    assert np.array_equal(w[:, :, :-1], lab[:, :, 1:]) and np.all(w[:, :, -1] == -1)
    d[2] = 0.5          # rounds half up
    assert np.array_equal(O.warp_labels_nearest(lab, d), w)


# ---------------------------------------------------------------------------
# One iteration and a small full run
# ---------------------------------------------------------------------------

def test_iteration_moves_at_most_eta_over_two_before_smoothing():
    n = (10, 11, 12)
    from paper_2404_01249_amd import synth
    p = synth.blobs_pair(n, seed=35, n_blobs=6, sigma_range=(1.5, 3.0), field_max=1.5, field_sigma=3.0)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.0, window=3)
    d0 = np.zeros((3,) + n)
    d1, m, v, L, ex = O.iterate(p.fixed, p.moving, d0, d0, d0, 1, P)
    assert np.sqrt((d1 ** 2).sum(0)).max() == pytest.approx(0.25, rel=1e-12)
    assert np.allclose(ex["u"], d1)     # from the identity, phi o (id+u) = id+u


def test_small_registration_descends_and_stays_diffeomorphic():
    from paper_2404_01249_amd import synth
    p = synth.blobs_pair((20, 22, 24), seed=36, n_blobs=8, sigma_range=(2.0, 4.0), field_sigma=4.0, field_max=2.0)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
    d, losses, t = O.register(p.fixed, p.moving, [2.0, 1.0], [20, 15], P)
    assert t == 35 and len(losses) == 35
    assert losses[19] < losses[0] and losses[-1] < losses[20]
    assert O.singular_fraction(d) == 0.0
    J0 = O.lncc_forward(p.fixed, p.moving, 5, 1e-5)[1]
    J1 = O.lncc_forward(p.fixed, O.warp_image(p.moving, d), 5, 1e-5)[1]
    assert J1 < J0


def test_level_transition_carries_adam_state_and_step_count():
    """Section 4.5: the warp and the optimiser state are upsampled to the next
    level, and the step count continues.  Two levels at scale 1 have the same
    grid, where corner-aligned upsampling is exactly the identity (positions
    i (n-1)/(n-1) = i, rho = 1), so splitting a run into two levels must give
    the single-level run bitwise.  Resetting m, v or t at the transition would
    change every later iteration (checked below by planting each reset)."""
    from paper_2404_01249_amd import synth
    p = synth.blobs_pair((9, 10, 11), seed=37, n_blobs=5, sigma_range=(1.5, 3.0), field_sigma=3.0, field_max=1.5)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=3)
    d1, l1, t1 = O.register(p.fixed, p.moving, [1.0], [7], P)
    d2, l2, t2 = O.register(p.fixed, p.moving, [1.0, 1.0], [3, 4], P)
    assert t1 == t2 == 7
    assert np.array_equal(d1, d2)
    assert np.array_equal(np.asarray(l1), np.asarray(l2))

    # the pin has power: each planted reset moves the result
    real_up, real_iter = O.fireants64.upsample_state, O.fireants64.iterate

    def reset_moments(d, m, v, shape_f):
        d, m, v = real_up(d, m, v, shape_f)
        return d, np.zeros_like(m), np.zeros_like(v)

    calls = {"n": 0}

    def restart_t(fixed, moving, d, m, v, t, P_):
        calls["n"] += 1
        return real_iter(fixed, moving, d, m, v, t if calls["n"] <= 3 else t - 3, P_)

    for name, fn in (("upsample_state", reset_moments), ("iterate", restart_t)):
        setattr(O.fireants64, name, fn)
        try:
            d3, _, _ = O.register(p.fixed, p.moving, [1.0, 1.0], [3, 4], P)
        finally:
            setattr(O.fireants64, "upsample_state", real_up)
            setattr(O.fireants64, "iterate", real_iter)
        assert np.abs(d3 - d1).max() > 1e-6, name
