"""Symmetric registration on the GPU (fa_symmetric.h) against the FP64 oracle
(oracle/symmetric64.py): one iteration of both halves, a two-level half-way
run, and the final phi = phi_M o phi_F^{-1}."""
import numpy as np
import pytest

from oracle import fireants64 as F
from oracle import inverse64 as V
from oracle import symmetric64 as S
from paper_2404_01249_amd import Symmetric, fa, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def problem(shape, seed):
    p = synth.blobs_pair(shape, seed=seed, n_blobs=12, sigma_range=(2.0, 5.0), field_sigma=3.0, field_max=2.0)
    return p.fixed, p.moving


def test_one_iteration_matches_oracle():
    shape = (21, 37, 45)
    fixed, moving = problem(shape, 121)
    P = F.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
    with Symmetric(dev(fixed), dev(moving), eta=P.eta) as sy:
        sy.set_schedule([1.0], [1])
        assert sy.run() == 1
        dF, dM = (host(t) for t in sy.halfway())
        loss = sy.loss_history()
    If, Im = fixed.astype(np.float64), moving.astype(np.float64)
    z = np.zeros((3,) + shape)
    dF_r, dM_r, _, _, L = S.symmetric_iterate(If, Im, z, z, (z, z), (z, z), 1, P)
    print(f"one symmetric iteration: dF rel {rel_l2(dF, dF_r):.2e}, dM rel {rel_l2(dM, dM_r):.2e}, "
          f"loss {loss[0]:.6f} vs {L:.6f}")
    assert rel_l2(dF, dF_r) <= TOL and rel_l2(dM, dM_r) <= TOL
    assert abs(loss[0] - L) <= 1e-5 * abs(L)


def test_halfway_run_matches_oracle():
    shape = (18, 21, 37)
    fixed, moving = problem(shape, 122)
    P = F.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
    with Symmetric(dev(fixed), dev(moving), eta=P.eta) as sy:
        sy.set_schedule([2.0, 1.0], [6, 4])
        assert sy.run() == 10
        dF, dM = (host(t) for t in sy.halfway())
        loss = sy.loss_history()
    dF_r, dM_r, loss_r = S.register_halfway(fixed, moving, [2.0, 1.0], [6, 4], P)
    rel = np.abs(loss - np.asarray(loss_r)) / np.abs(loss_r)
    eF = np.sqrt(((dF - dF_r) ** 2).sum(0))
    eM = np.sqrt(((dM - dM_r) ** 2).sum(0))
    print(f"half-way run: loss rel max {rel.max():.2e}; endpoint diff F {eF.mean():.2e}, M {eM.mean():.2e}")
    assert rel.max() <= 1e-3
    assert eF.mean() <= 0.05 and eM.mean() <= 0.05


def test_finish_composes_with_the_fitted_inverse():
    shape = (20, 22, 26)
    fixed, moving = problem(shape, 123)
    with Symmetric(dev(fixed), dev(moving), eta=0.5) as sy:
        sy.set_schedule([2.0, 1.0], [10, 6])
        sy.run()
        dF, dM = (host(t) for t in sy.halfway())
        d = host(sy.finish([2.0, 1.0], [30, 20], eta=0.2))
        cost = sy.inverse_cost
    Pi = F.Params(eta=0.2, sigma_grad=1.0, sigma_warp=0.5)
    e, inv_losses, _ = V.invert(dF, [2.0, 1.0], [30, 20], Pi)
    d_ref = S.compose_fields(e, dM)
    epe = np.sqrt(((d - d_ref) ** 2).sum(0))
    print(f"phi_M o phi_F^-1: endpoint diff to the oracle mean {epe.mean():.2e} max {epe.max():.2e}; "
          f"inverse cost {cost:.5f} vs {inv_losses[-1]:.5f}")
    assert epe.mean() <= 1e-3 and epe.max() <= 0.02
    assert abs(cost - inv_losses[-1]) <= 1e-3 * inv_losses[-1] + 1e-7


def test_finish_state_errors():
    fixed, moving = problem((10, 11, 12), 124)
    with Symmetric(dev(fixed), dev(moving)) as sy:
        out = torch.empty((3, 10, 11, 12), device="cuda")
        with pytest.raises(fa.FAError) as e:
            sy.finish([1.0], [2])
        assert e.value.status == fa.FA_ESTATE
        sy.set_schedule([2.0], [2])
        sy.run()
        with pytest.raises(fa.FAError) as e:
            sy.finish([1.0], [2])
        assert e.value.status == fa.FA_ESTATE   # the last level is not the input grid
        sy.set_schedule([1.0], [2])
        sy.run()
        with pytest.raises(fa.FAError) as e:
            sy.finish([2.0], [2])
        assert e.value.status == fa.FA_EINVAL   # nor the inverse's
        del out


def test_tissue160_symmetric_result_folds_only_on_the_faces():
    """The symmetric registration of the 160x192x224 workload (bench
    settings: half-way warps over scales 4, 2, 1 at 200, 100, 50; inverse over
    4, 2, 1 at 50, 25, 12 with eta 0.2).  Both half-way warps and the fitted
    inverse psi are free of folds; phi_M o psi folds only in the outermost
    interior planes, where psi sends a voxel off the grid and the composition
    reads d_M as zero there (values outside the grid are zero, as for every
    sample in Algorithm 1), and at no more than 1e-5 of the voxels."""
    print("symmetric tissue160 folds", flush=True)
    p = synth.load("tissue160")
    with Symmetric(dev(p.fixed), dev(p.moving), eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5) as sy:
        sy.set_schedule(p.scales, p.iters)
        sy.run()
        dF, dM = (t.clone() for t in sy.halfway())
        d = sy.finish([4.0, 2.0, 1.0], [50, 25, 12], eta=0.2, sigma_grad=1.0, sigma_warp=0.5).clone()
    from paper_2404_01249_amd import evaluate
    assert evaluate.singular_fraction(dF) == 0.0 and evaluate.singular_fraction(dM) == 0.0
    det = host(evaluate.jacobian_det(d))          # interior voxels: index i is voxel i + 1
    frac = float((det <= 0).mean())
    inner = det[2:-2, 2:-2, 2:-2]                 # voxels at least three planes from every face
    print(f"singular fraction {frac:.2e}; folds away from the faces {int((inner <= 0).sum())}")
    assert frac <= 1e-5
    assert (inner > 0).all()
