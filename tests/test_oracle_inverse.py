"""Pins of the post hoc inverse oracle (oracle/inverse64.py) against what the
mathematics fixes, independently of the oracle's own formulas:

* the splat is the adjoint of trilinear sampling (an inner-product identity)
  and is the identity at the grid nodes;
* the gradient matches central differences of the cost;
* d = 0 gives U = 2 mean |e|^2 and dU/de = 4 e / N in closed form;
* an affine warp's exact inverse (a matrix inverse) zeroes both residuals and
  the gradient away from the faces;
* the fitted inverse of a smooth warp agrees with the classical fixed-point
  inverse e(y) = -d(y + e(y)), a different method;
* downsampling keeps constant fields (divided by rho) and linear fields.
"""
import numpy as np
import pytest

from oracle import fireants64 as F
from oracle import inverse64 as V



def test_splat_is_the_adjoint_of_trilinear_sampling():
    rng = np.random.default_rng(1)
    shape = (6, 7, 8)
    f = rng.standard_normal(shape)
    pts = (50,)
    p = np.stack([rng.uniform(-1.5, n + 0.5, pts) for n in shape])   # some samples off the grid
    w = rng.standard_normal(pts)
    lhs = float((F.trilinear(f, p) * w).sum())
    rhs = float((f * V.splat(w, p, shape)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_splat_at_nodes_and_at_one_point():
    rng = np.random.default_rng(2)
    shape = (4, 5, 6)
    w = rng.standard_normal(shape)
    assert np.array_equal(V.splat(w, F.identity_grid(shape), shape), w)
    out = V.splat(np.array([1.0]), np.array([[1.25], [2.5], [3.75]]), shape)
    # weights (1 - t) or t per axis: t = 0.25, 0.5, 0.75
    assert out[1, 2, 3] == pytest.approx(0.75 * 0.5 * 0.25)
    assert out[2, 3, 4] == pytest.approx(0.25 * 0.5 * 0.75)
    assert out.sum() == pytest.approx(1.0)
    # a sample beyond the last node keeps only the weights of in-grid nodes
    out = V.splat(np.array([1.0]), np.array([[3.5], [0.0], [0.0]]), shape)
    assert out.sum() == pytest.approx(0.5)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)
    d = rng.uniform(-1.2, 1.2, (3,) + shape)
    e = rng.uniform(-0.8, 0.8, (3,) + shape)
    g, U = V.inverse_gradient(d, e)
    assert U == pytest.approx(V.inverse_cost(d, e), rel=1e-14)
    h = 1e-6
    for _ in range(25):
        c = int(rng.integers(0, 3))
        j = tuple(int(rng.integers(0, n)) for n in shape)
        ep, em = e.copy(), e.copy()
        ep[(c,) + j] += h
        em[(c,) + j] -= h
        fd = (V.inverse_cost(d, ep) - V.inverse_cost(d, em)) / (2 * h)
        assert g[(c,) + j] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_zero_warp_closed_form():
    rng = np.random.default_rng(4)
    shape = (5, 4, 6)
    e = rng.uniform(-1.0, 1.0, (3,) + shape)
    g, U = V.inverse_gradient(np.zeros_like(e), e)
    N = float(np.prod(shape))
    assert U == pytest.approx(2.0 * (e * e).sum() / N, rel=1e-14)
    np.testing.assert_allclose(g, 4.0 * e / N, rtol=1e-13, atol=1e-16)


def test_affine_warp_exact_inverse():
    shape = (12, 13, 14)
    A = np.array([[0.04, -0.03, 0.02], [0.05, -0.02, 0.01], [-0.01, 0.03, 0.06]])
    b = np.array([0.3, -0.2, 0.4])
    X = F.identity_grid(shape)
    d = np.einsum("ij,j...->i...", A, X) + b[:, None, None, None]
    inv = np.linalg.inv(np.eye(3) + A)
    e = np.einsum("ij,j...->i...", inv, X - b[:, None, None, None]) - X
    r1, r2, _, _ = V.inverse_residuals(d, e)
    g, _ = V.inverse_gradient(d, e)
    core = tuple(slice(3, n - 3) for n in shape)
    deep = tuple(slice(5, n - 5) for n in shape)
    assert np.abs(r1[(slice(None),) + core]).max() < 1e-12
    assert np.abs(r2[(slice(None),) + core]).max() < 1e-12
    assert np.abs(g[(slice(None),) + deep]).max() < 1e-14
    # a wrong inverse (the first-order guess -d) leaves a residual
    r1w, _, _, _ = V.inverse_residuals(d, -d)
    assert np.abs(r1w[(slice(None),) + core]).max() > 1e-3


def fixed_point_inverse(d, iters=60):
    """e(y) = -d(y + e(y)) by fixed-point iteration (converges for
    |grad d| < 1)."""
    X = F.identity_grid(d.shape[1:])
    e = -d.copy()
    for _ in range(iters):
        e = -np.stack([F.trilinear(d[c], X + e) for c in range(3)])
    return e


def test_fitted_inverse_matches_the_fixed_point_inverse():
    shape = (20, 22, 24)
    d = F.gaussian_smooth(np.random.default_rng(5).standard_normal((3,) + shape), 3.0)
    d *= 1.5 / np.sqrt((d * d).sum(0)).max()
    # every step moves psi by eta/2 at its largest, so eta bounds how close
    # the iterates settle: a small eta for a tight comparison
    P = F.Params(eta=0.1, sigma_grad=1.0, sigma_warp=0.5)
    e, losses, t = V.invert(d, [2.0, 1.0], [100, 100], P)
    assert t == 200 and len(losses) == 200
    ref = fixed_point_inverse(d)
    core = (slice(None),) + tuple(slice(4, n - 4) for n in shape)
    err = np.sqrt(((e - ref)[core] ** 2).sum(0))
    assert err.mean() < 0.002 and err.max() < 0.01, (err.mean(), err.max())
    r1, r2, _, _ = V.inverse_residuals(d, e)
    assert np.sqrt((r1[core] ** 2).sum(0)).max() < 0.01
    assert np.sqrt((r2[core] ** 2).sum(0)).max() < 0.01
    # near the faces the zero extension leaves a residual no inverse removes;
    # the fit does at least as well there as the fixed point
    assert losses[-1] <= V.inverse_cost(d, ref)
    assert losses[-1] < 0.2 * losses[0]


def test_downsample_field_constants_and_linear_fields():
    shape = (17, 21, 25)
    c = np.array([0.7, -1.1, 2.0])
    d = np.broadcast_to(c[:, None, None, None], (3,) + shape).copy()
    dc = V.downsample_field(d, 2.0)
    shp_c = F.level_shape(shape, 2.0)
    rho = [(shape[a] - 1) / (shp_c[a] - 1) for a in range(3)]
    for a in range(3):
        np.testing.assert_allclose(dc[a], c[a] / rho[a], rtol=1e-13)
    X = F.identity_grid(shape)
    lin = 0.05 * X   # phi = 1.05 x: the same map in coarse voxel units
    dl = V.downsample_field(lin, 2.0)
    Xc = F.identity_grid(shp_c)
    core = (slice(None),) + tuple(slice(3, n - 3) for n in shp_c)
    np.testing.assert_allclose(dl[core], 0.05 * Xc[core], rtol=1e-12, atol=1e-12)
    assert np.array_equal(V.downsample_field(d, 1.0), d)


def test_zero_warp_keeps_the_identity():
    d = np.zeros((3, 6, 7, 8))
    e, losses, _ = V.invert(d, [1.0], [3], F.Params())
    assert np.array_equal(e, np.zeros_like(d)) and losses == [0.0, 0.0, 0.0]
