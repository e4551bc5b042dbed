"""Evaluation kernels (include/fa_eval.h) against the oracle: label transfer
and overlap counts bit for bit, det(I + grad d) bit for bit (both sides
evaluate it in double precision in the same order), and a whole 160x192x224
registration against the stored oracle run (field, Dice, singular fraction).
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_01249_amd import Pair, evaluate, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def dev(x, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def labels_and_field(shape, seed, scale=3.0):
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 4, size=shape).astype(np.int8)
    d = synth.smooth_field(shape, seed, sigma=2.0, max_norm=scale)
    # exact half-integers (round half up), their neighbours and far / non-finite values
    flat = d.reshape(3, -1)
    k = rng.integers(0, flat.shape[1], size=200)
    flat[:, k[:50]] = np.float32(0.5)
    flat[:, k[50:100]] = np.float32(-1.5)
    flat[:, k[100:150]] = np.nextafter(np.float32(0.5), np.float32(0.0))
    flat[0, k[150:170]] = np.float32(1e12)
    flat[1, k[170:180]] = np.float32(-7.0e9)
    flat[2, k[180:190]] = np.float32(np.nan)
    flat[2, k[190:200]] = np.float32(-np.inf)
    return lab, d


@pytest.mark.parametrize("shape", [(21, 37, 45), (7, 5, 6), (2, 3, 130)])
def test_warp_labels_exact(shape):
    print(f"warp_labels {shape}", flush=True)
    lab, d = labels_and_field(shape, seed=31)
    with np.errstate(invalid="ignore"):
        ref = O.warp_labels_nearest(lab, d.astype(np.float64))
    got = host(evaluate.warp_labels(dev(lab, np.int8), dev(d))).astype(np.int64)
    assert np.array_equal(got, ref)
    # identity transfers every label
    zero = np.zeros((3,) + shape, np.float32)
    assert np.array_equal(host(evaluate.warp_labels(dev(lab, np.int8), dev(zero))), lab)


@pytest.mark.parametrize("n,n_classes", [(0, 4), (1, 4), (1000, 4), (3_000_001, 7), (257, 127)])
def test_label_overlap_and_dice_exact(n, n_classes):
    rng = np.random.default_rng(n + n_classes)
    a = rng.integers(-1, n_classes + 1, size=n).astype(np.int8)
    b = np.where(rng.random(n) < 0.7, a, rng.integers(-1, n_classes + 1, size=n)).astype(np.int8)
    got = evaluate.label_overlap(dev(a, np.int8), dev(b, np.int8), n_classes)
    ref = np.array([[(a == r).sum(), (b == r).sum(), ((a == r) & (b == r)).sum()] for r in range(n_classes)])
    assert np.array_equal(got, ref)
    if n:
        assert evaluate.dice(dev(a, np.int8), dev(b, np.int8), n_classes) == O.dice(a, b, range(n_classes))


@pytest.mark.parametrize("shape", [(21, 37, 45), (3, 3, 3), (5, 4, 131)])
def test_jacobian_det_exact(shape):
    print(f"jacobian_det {shape}", flush=True)
    rng = np.random.default_rng(41)
    d = synth.smooth_field(shape, 41, sigma=1.0, max_norm=2.5)       # rough enough to fold
    d += rng.normal(0.0, 0.3, size=d.shape).astype(np.float32)
    ref = O.jacobian_det(d)
    got = host(evaluate.jacobian_det(dev(d)))
    assert got.dtype == np.float64 and got.shape == ref.shape
    assert np.array_equal(got, ref)
    assert evaluate.singular_fraction(dev(d)) == O.singular_fraction(d)
    if shape == (21, 37, 45):
        assert 0.0 < O.singular_fraction(d) < 1.0     # the case exercises both signs


def test_jacobian_det_without_interior():
    d = np.zeros((3, 2, 5, 6), np.float32)
    assert evaluate.jacobian_det(dev(d)).numel() == 0
    assert np.isnan(evaluate.singular_fraction(dev(d)))


@pytest.mark.parametrize("shape", [(21, 37, 45), (7, 5, 6)])
def test_compose_fields_matches_oracle(shape):
    """u + d(x + u) against the oracle's composition (fp64), with samples off
    the grid near the faces."""
    u = synth.smooth_field(shape, 61, sigma=2.0, max_norm=3.0)
    d = synth.smooth_field(shape, 62, sigma=2.0, max_norm=2.0)
    got = host(evaluate.compose(dev(u), dev(d))).astype(np.float64)
    ref = O.compose(d.astype(np.float64), u.astype(np.float64))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"{shape}: compose max rel {err:.2e}")
    assert err <= 1e-6
    # composing with a zero field is exact
    z = np.zeros_like(u)
    assert np.array_equal(host(evaluate.compose(dev(u), dev(z))), u)
    assert np.array_equal(host(evaluate.compose(dev(z), dev(d))), d)


def test_tissue160_registration_matches_stored_oracle_run():
    """The whole 160x192x224 schedule (4x, 2x, 1x at 200/100/50) against the
    oracle's run stored by tests/golden/make_golden.py."""
    print("tissue160 full run", flush=True)
    z = np.load(os.path.join(HERE, "golden", "tissue160_oracle.npz"))
    p = synth.load("tissue160")
    pr = Pair(dev(p.fixed), dev(p.moving), eta=float(z["eta"]), sigma_grad=float(z["sigma_grad"]),
              sigma_warp=float(z["sigma_warp"]), window=int(z["window"]))
    pr.set_schedule(list(z["scales"]), list(z["iters"]))
    pr.run()
    loss = pr.loss_history().astype(np.float64)
    d = pr.field()
    s = int(z["field_stride"])
    dh = host(d).astype(np.float64)[:, ::s, ::s, ::s]
    epe = float(np.sqrt(((dh - z["field"]) ** 2).sum(0)).mean())
    rel = np.abs(loss - z["losses"]) / np.abs(z["losses"])
    warped = evaluate.warp_labels(dev(p.moving_labels, np.int8), d)
    dsc = evaluate.dice(warped, dev(p.fixed_labels, np.int8), 4)
    sing = evaluate.singular_fraction(d)
    print(f"tissue160: endpoint diff {epe:.4f} vox, loss rel first {rel[0]:.2e} max {rel.max():.2e}, "
          f"Dice {dsc:.4f} (oracle {float(z['dice']):.4f}, identity {float(z['dice_identity']):.4f}), "
          f"singular {sing:.2e}", flush=True)
    # the distance by which the result misses the warp that made the moving image
    miss, miss_max = evaluate.endpoint_error(d, dev(p.true_field))
    miss_id, _ = evaluate.endpoint_error(torch.zeros_like(d), dev(p.true_field))
    print(f"tissue160: endpoint error against the true warp {miss:.3f} vox (max {miss_max:.2f}); "
          f"identity {miss_id:.3f}", flush=True)
    assert epe <= 0.05
    assert rel[0] <= 1e-5 and rel.max() <= 1e-2
    assert abs(dsc - float(z["dice"])) <= 0.005
    assert sing == float(z["singular"]) == 0.0
    assert miss < 0.5 * miss_id
    pr.close()
