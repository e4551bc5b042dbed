"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Every case feeds the same seeded float32 inputs to the library and (promoted
to float64) to the oracle, then compares element by element.  Tolerances
(relative, each defined as below):

* warped intensity: max|dJ| / max|J|  <= 1e-5
* loss:             |dL| / |L|        <= 1e-5
* gradients and the quantities computed from them (Adam moments and
  direction, smoothed steps, updated displacement): ||d||_2 / ||ref||_2 <= 1e-4
* full run: mean endpoint difference <= 0.05 voxel

Shapes span several in-plane tiles with ragged tails in both tiled axes, and
n0 chunks with a ragged last chunk.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_01249_amd import Pair, fa, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_J = 1e-5
TOL_L = 1e-5
TOL_G = 1e-4


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def make_problem(shape, seed, field_max=2.0):
    p = synth.blobs_pair(shape, seed=seed, n_blobs=12, sigma_range=(2.0, 5.0), field_sigma=3.0,
                         field_max=field_max)
    d = synth.smooth_field(shape, seed + 1000, sigma=3.0, max_norm=1.5)
    return p.fixed, p.moving, d


def new_pair(fixed, moving, **kw):
    pr = Pair(dev(fixed), dev(moving), **kw)
    return pr


def check_run_against_oracle(loss, d, d_ref, loss_ref, label=""):
    """The run tolerances of a registration against the oracle (loss history
    and final field; see test_random_configurations_match_oracle)."""
    rel = np.abs(np.asarray(loss, np.float64) - np.asarray(loss_ref)) / np.maximum(np.abs(loss_ref), 1e-12)
    epe = np.sqrt(((d - d_ref) ** 2).sum(0))
    q = float(np.quantile(epe, 0.999))
    print(f"{label}: loss rel max {rel.max():.2e}, endpoint diff mean {epe.mean():.2e} 99.9% {q:.2e}")
    assert rel[0] <= 1e-5 and rel.max() <= 1e-3, label
    assert epe.mean() <= 1e-3 and q <= 0.05, label


SHAPES = [(21, 37, 45), (12, 131, 133), (7, 5, 6)]


@pytest.mark.parametrize("shape", SHAPES)
def test_warp_identity_shift_and_random(shape):
    fixed, moving, d = make_problem(shape, seed=11)
    pr = new_pair(fixed, moving)
    pr.set_schedule([1.0], [1])
    zero = np.zeros((3,) + shape, np.float32)
    pr.set_state(dev(zero), None, None, 0)
    assert np.array_equal(host(pr.warped()), moving.astype(np.float64))          # identity: bitwise
    shift = np.zeros_like(zero)
    shift[0], shift[1], shift[2] = 1.0, -2.0, 3.0
    pr.set_state(dev(shift), None, None, 0)
    ref = O.warp_image(moving, shift)
    assert np.array_equal(host(pr.warped()), ref)                                 # integer shift: exact
    pr.set_state(dev(d), None, None, 0)
    ref = O.warp_image(moving, d)
    got = host(pr.warped())
    assert np.abs(got - ref).max() / np.abs(ref).max() <= TOL_J
    pr.close()


# gradient kernel forms: 1 = the march along n0, 3 = bricks (windows 1 to 5;
# the automatic choice for volumes up to 300,000 voxels)
GRAD_FORMS = [1, 3]


@pytest.mark.parametrize("form", GRAD_FORMS)
@pytest.mark.parametrize("window", [1, 3, 5, 7, 9])
@pytest.mark.parametrize("shape", SHAPES)
def test_gradient_and_loss_match_oracle(shape, window, form):
    fixed, moving, d = make_problem(shape, seed=21 + window)
    pr = new_pair(fixed, moving, window=window)
    fa.fa_pair_set_tuning(pr.handle, 0, 0, 0, 0, form)
    pr.set_schedule([1.0], [1])
    pr.set_state(dev(d), None, None, 0)
    g, loss = pr.eval_gradient()
    g_ref, L_ref = O.gateaux_gradient(fixed, moving, d, window, 1e-5)
    assert abs(loss - L_ref) <= TOL_L * abs(L_ref)
    assert rel_l2(host(g), g_ref) <= TOL_G
    pr.close()


@pytest.mark.parametrize("form", GRAD_FORMS)
@pytest.mark.parametrize("shape", [(21, 37, 45), (12, 131, 133)])
def test_one_iteration_from_injected_state(shape, form):
    """Every intermediate of one iteration of Algorithm 1 from the same state."""
    fixed, moving, d = make_problem(shape, seed=31)
    rng = np.random.default_rng(32)
    m = (1e-6 * rng.standard_normal((3,) + shape)).astype(np.float32)
    v = (1e-12 * rng.random((3,) + shape)).astype(np.float32)
    t_done = 7
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
    pr = new_pair(fixed, moving, eta=P.eta, sigma_grad=P.sigma_grad, sigma_warp=P.sigma_warp, window=5)
    fa.fa_pair_set_tuning(pr.handle, 0, 0, 0, 0, form)
    pr.set_schedule([1.0], [1])
    pr.set_state(dev(d), dev(m), dev(v), t_done)
    pr.step(1)
    d1, m1, v1 = (host(x) for x in pr.state())
    a = host(pr.direction())
    M = pr.step_norm()
    loss = pr.loss_history()
    ref_d, ref_m, ref_v, ref_L, ex = O.iterate(fixed, moving, d.astype(np.float64), m.astype(np.float64),
                                               v.astype(np.float64), t_done + 1, P)
    assert len(loss) == 1
    assert abs(loss[-1] - ref_L) <= TOL_L * abs(ref_L)
    assert rel_l2(m1, ref_m) <= TOL_G
    assert rel_l2(v1, ref_v) <= TOL_G
    assert rel_l2(a, ex["a"]) <= TOL_G
    assert abs(M - ex["M"]) <= TOL_G * ex["M"]
    assert rel_l2(d1 - d, ref_d - d) <= TOL_G       # the update itself, not just d
    assert np.abs(d1 - ref_d).max() <= 1e-4
    pr.close()


@pytest.mark.parametrize("form", GRAD_FORMS)
def test_one_iteration_with_use_jac(form):
    """Algorithm 1 with use_jac: the Eulerian direction J(phi)^T g (Section
    4.4.2) replaces the Gateaux gradient before Adam.  The displacement has
    gradients of order 0.5, so the Jacobian term is far from negligible."""
    shape = (21, 37, 45)
    fixed, moving, _ = make_problem(shape, seed=37)
    d = synth.smooth_field(shape, 38, sigma=2.0, max_norm=2.5)
    rng = np.random.default_rng(39)
    m = (1e-6 * rng.standard_normal((3,) + shape)).astype(np.float32)
    v = (1e-12 * rng.random((3,) + shape)).astype(np.float32)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5, use_jac=True)
    pr = new_pair(fixed, moving, eta=P.eta, sigma_grad=P.sigma_grad, sigma_warp=P.sigma_warp, window=5,
                  use_jac=True)
    fa.fa_pair_set_tuning(pr.handle, 0, 0, 0, 0, form)
    pr.set_schedule([1.0], [1])
    pr.set_state(dev(d), dev(m), dev(v), 4)
    pr.step(1)
    d1, m1, v1 = (host(x) for x in pr.state())
    a = host(pr.direction())
    ref_d, ref_m, ref_v, ref_L, ex = O.iterate(fixed, moving, d.astype(np.float64), m.astype(np.float64),
                                               v.astype(np.float64), 5, P)
    g_plain, _ = O.gateaux_gradient(fixed, moving, d, 5, 1e-5)
    assert rel_l2(O.eulerian_direction(g_plain, d), g_plain) > 0.05     # the term matters here
    assert abs(pr.loss_history()[-1] - ref_L) <= TOL_L * abs(ref_L)
    assert rel_l2(m1, ref_m) <= TOL_G
    assert rel_l2(v1, ref_v) <= TOL_G
    assert rel_l2(a, ex["a"]) <= TOL_G
    assert abs(pr.step_norm() - ex["M"]) <= TOL_G * ex["M"]
    assert rel_l2(d1 - d, ref_d - d) <= TOL_G
    pr.close()


def test_short_run_with_use_jac_matches_oracle():
    shape = (21, 37, 45)
    fixed, moving, _ = make_problem(shape, seed=40, field_max=2.5)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5, use_jac=True)
    pr = new_pair(fixed, moving, window=5, use_jac=True)
    pr.set_schedule([2.0, 1.0], [8, 6])
    pr.run()
    loss = pr.loss_history().astype(np.float64)
    d = host(pr.field())
    d_ref, loss_ref, _ = O.register(fixed, moving, [2.0, 1.0], [8, 6], P)
    rel = np.abs(loss - np.asarray(loss_ref)) / np.abs(np.asarray(loss_ref))
    epe = float(np.sqrt(((d - d_ref) ** 2).sum(0)).mean())
    print(f"use_jac run: loss rel max {rel.max():.2e}, mean endpoint diff {epe:.2e}", flush=True)
    assert rel.max() <= 1e-4
    assert epe <= 1e-3
    pr.close()


@pytest.mark.parametrize("eta,sigma_grad,sigma_warp", [(2.0, 0.3, 0.0), (3.0, 0.5, 1.0), (0.25, 0.0, 0.4),
                                                      (1.0, 2.0, 2.0), (0.25, 6.0, 0.4), (1.0, 2.5, 3.0),
                                                      (3.0, 8.0, 7.5)])
def test_one_iteration_step_variants(eta, sigma_grad, sigma_warp):
    """Both composition paths (staged in LDS for eta <= 2, gathered beyond)
    and Gaussian radii 0..24, from an injected state: radii up to 6 run the
    streaming kernels, wider ones (sigma_grad 6 and sigma_warp 0.4 are the
    lung CT settings of the paper's EMPIRE10 runs) the separable passes with
    a run-time radius, which here exceed every axis of the volume."""
    shape = (19, 33, 41)
    fixed, moving, d = make_problem(shape, seed=33)
    P = O.Params(eta=eta, sigma_grad=sigma_grad, sigma_warp=sigma_warp, window=3)
    pr = new_pair(fixed, moving, eta=eta, sigma_grad=sigma_grad, sigma_warp=sigma_warp, window=3)
    pr.set_schedule([1.0], [1])
    pr.set_state(dev(d), None, None, 0)
    pr.step(1)
    d1 = host(pr.state()[0])
    z = np.zeros((3,) + shape)
    ref_d, _, _, ref_L, ex = O.iterate(fixed, moving, d.astype(np.float64), z, z, 1, P)
    assert rel_l2(d1 - d, ref_d - d) <= TOL_G
    assert abs(pr.step_norm() - ex["M"]) <= TOL_G * ex["M"]
    assert abs(pr.loss_history()[-1] - ref_L) <= TOL_L * abs(ref_L)
    pr.close()


@pytest.mark.parametrize("shape", [(21, 37, 45), (40, 48, 56)])
def test_run_with_lung_ct_smoothing_matches_oracle(shape):
    """A two-level run with the paper's EMPIRE10 hyperparameters (eta 0.25,
    sigma_grad 6, sigma_warp 0.4; Datasets and Evaluation Metrics, lung CT)
    against the oracle: the radius-18 smoothing of the direction runs the
    wide passes at both levels, the radius-2 warp smoothing the streaming or
    brick kernels."""
    fixed, moving, _ = make_problem(shape, seed=34)
    kw = dict(eta=0.25, sigma_grad=6.0, sigma_warp=0.4, window=5)
    scales, iters = [2.0, 1.0], [6, 4]
    pr = new_pair(fixed, moving, **kw)
    pr.set_schedule(scales, iters)
    assert pr.run() == sum(iters)
    loss, d = pr.loss_history(), host(pr.field())
    pr.close()
    d_ref, loss_ref, _ = O.register(fixed, moving, scales, iters, O.Params(**kw))
    check_run_against_oracle(loss, d, d_ref, loss_ref, label=f"lung CT smoothing {shape}")


@pytest.mark.parametrize("shape,sigma_grad,sigma_warp,eta", [((21, 37, 45), 1.0, 0.5, 0.5), ((40, 48, 56), 0.3, 0.0, 2.0),
                                                           ((7, 5, 6), 0.0, 1.0, 1.0), ((13, 17, 33), 0.9, 0.9, 0.25)])
def test_brick_launches_match_streaming_launches(shape, sigma_grad, sigma_warp, eta):
    """The brick (whole-in-LDS) forms of the smoothing and composition kernels
    give bitwise the results of the streaming forms (radii 0 to 3)."""
    fixed, moving, _ = make_problem(shape, seed=36)
    out = []
    for variant in (1, 2):
        pr = new_pair(fixed, moving, eta=eta, sigma_grad=sigma_grad, sigma_warp=sigma_warp, window=5)
        for kind in (1, 2, 3):
            fa.fa_pair_set_tuning(pr.handle, kind, 0, 0, 0, variant)
        pr.set_schedule([1.0], [6])
        pr.run()
        out.append((pr.loss_history(), host(pr.field()), pr.step_norm()))
        pr.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


@pytest.mark.parametrize("shape", [(21, 37, 45), (13, 17, 33)])
def test_loss_record_in_either_launch(shape):
    """The iteration's loss record and step count run in the composition, or in
    the warp smoothing when that is a brick launch: every mix of brick and
    streaming forms for the two (the autotuner may pick any) gives bitwise the
    same loss history, field and step norm."""
    fixed, moving, _ = make_problem(shape, seed=37)
    out = []
    for warp, compose in ((1, 1), (2, 1), (1, 2), (2, 2)):   # 1 streaming, 2 brick
        pr = new_pair(fixed, moving, eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=5)
        fa.fa_pair_set_tuning(pr.handle, 2, 0, 0, 0, warp)      # kind 2: warp smoothing
        fa.fa_pair_set_tuning(pr.handle, 3, 0, 0, 0, compose)   # kind 3: composition
        pr.set_schedule([2.0, 1.0], [4, 5])
        assert pr.tiling(1, 2)[3] == (warp == 2) and pr.tiling(1, 3)[3] == (compose == 2)
        pr.run()
        out.append((pr.loss_history(), host(pr.field()), pr.step_norm()))
        pr.close()
    assert len(out[0][0]) == 9
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0])
        assert np.array_equal(out[0][1], o[1])
        assert out[0][2] == o[2]


def test_first_iteration_moves_at_most_eta_over_two():
    fixed, moving, _ = make_problem((21, 37, 45), seed=41)
    pr = new_pair(fixed, moving, eta=0.5, sigma_grad=1.0, sigma_warp=0.0)
    pr.set_schedule([1.0], [1])
    pr.step(1)
    d = host(pr.field())
    assert np.sqrt((d ** 2).sum(0)).max() == pytest.approx(0.25, rel=1e-5)
    pr.close()


# Blur radii ceil(3 s / 2), applied at full resolution: 6 and 3; 3; 5 and 3;
# 8 (the one-output-per-thread form), 4 and 2; 6, 4 and 2.  Most of these n0
# and n1 end in a partial run of eight outputs.
@pytest.mark.parametrize("shape,scales", [((48, 56, 40), [4.0, 2.0, 1.0]), ((23, 19, 37), [2.0, 1.0]),
                                          ((33, 64, 70), [3.0, 1.5]), ((40, 44, 52), [5.0, 2.5, 1.2]),
                                          ((29, 21, 37), [4.0, 2.5, 1.2])])
def test_pyramid_levels_match_oracle(shape, scales):
    p = synth.tissue_pair(shape, seed=51, bias_sigma=6.0, field_sigma=4.0, field_max=2.0)
    pr = new_pair(p.fixed, p.moving)
    pr.set_schedule(scales, [1] * len(scales))
    for lvl, s in enumerate(scales):
        for which, img in ((0, p.fixed), (1, p.moving)):
            got = host(pr.level_image(lvl, which))
            ref = O.downsample_image(img, s)
            assert got.shape == ref.shape == O.level_shape(shape, s)
            assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    pr.close()


def test_level_transition_upsamples_state():
    shape = (24, 30, 34)
    fixed, moving, _ = make_problem(shape, seed=61)
    pr = new_pair(fixed, moving)
    pr.set_schedule([2.0, 1.0], [0, 0])
    cshape = O.level_shape(shape, 2.0)
    rng = np.random.default_rng(62)
    d = synth.smooth_field(cshape, 63, sigma=2.0, max_norm=1.0)
    m = rng.standard_normal((3,) + cshape).astype(np.float32)
    v = rng.random((3,) + cshape).astype(np.float32)
    pr.set_state(dev(d), dev(m), dev(v), 3)
    done, fin = pr.step(1)
    assert done == 0 and fin == 1
    assert pr.progress()[0] == 1
    d2, m2, v2 = (host(x) for x in pr.state())
    rd, rm, rv = O.upsample_state(d.astype(np.float64), m.astype(np.float64), v.astype(np.float64), shape)
    for got, ref in ((d2, rd), (m2, rm), (v2, rv)):
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    pr.close()


def _full_run(name, form=0):
    p = synth.load(name)
    gold = np.load(os.path.join(HERE, "golden", f"{name}_oracle.npz"), allow_pickle=False)
    pr = new_pair(p.fixed, p.moving, eta=float(gold["eta"]), sigma_grad=float(gold["sigma_grad"]),
                  sigma_warp=float(gold["sigma_warp"]), window=int(gold["window"]))
    for kind in range(4):
        fa.fa_pair_set_tuning(pr.handle, kind, 0, 0, 0, form)
    pr.set_schedule(list(gold["scales"]), [int(i) for i in gold["iters"]])
    done = pr.run()
    assert done == int(np.sum(gold["iters"]))
    return p, gold, pr


@pytest.mark.parametrize("form", [0, 1])
def test_full_run_blobs64_matches_oracle(form):
    """Whole 64^3 two-level run against the stored oracle run, with the
    automatic kernel forms (bricks at both levels) and with every kernel
    marching along n0.  The bound is the mean endpoint difference (0.05
    voxel); the loss trajectory is also held close (fp32 and fp64
    trajectories separate slowly once the fixed-length steps of Appendix E
    oscillate around the optimum)."""
    p, gold, pr = _full_run("blobs64", form)
    loss = pr.loss_history().astype(np.float64)
    ref = gold["losses"]
    assert loss.shape == ref.shape
    s = int(gold["field_stride"])
    d = host(pr.field())[:, ::s, ::s, ::s]
    epe = float(np.sqrt(((d - gold["field"]) ** 2).sum(0)).mean())
    rel = np.abs(loss - ref) / np.abs(ref)
    print(f"full run: mean endpoint diff {epe:.4f} vox; loss rel diff first {rel[0]:.2e}, "
          f"level-0 max {rel[:100].max():.2e}, overall max {rel.max():.2e}")
    assert rel[0] <= TOL_L              # same state, same cost
    assert epe <= 0.05
    assert rel.max() <= 1e-2
    pr.close()


def test_full_run_microscopy128_matches_oracle():
    """Four-level run (8x, 4x, 2x, 1x at 40/20/10/5) with an LNCC window of
    7^3 on the microscopy-like recipe, against the stored oracle run."""
    p, gold, pr = _full_run("microscopy128")
    loss = pr.loss_history().astype(np.float64)
    ref = gold["losses"]
    s = int(gold["field_stride"])
    d = host(pr.field())[:, ::s, ::s, ::s]
    epe = float(np.sqrt(((d - gold["field"]) ** 2).sum(0)).mean())
    rel = np.abs(loss - ref) / np.abs(ref)
    print(f"microscopy128 run: mean endpoint diff {epe:.4f} vox; loss rel first {rel[0]:.2e}, "
          f"max {rel.max():.2e}", flush=True)
    assert rel[0] <= TOL_L
    assert epe <= 0.05
    assert rel.max() <= 1e-2
    pr.close()


def test_runs_are_bitwise_deterministic():
    fixed, moving, _ = make_problem((21, 37, 45), seed=71)
    hist = []
    for _ in range(2):
        pr = new_pair(fixed, moving)
        pr.set_schedule([2.0, 1.0], [6, 4])
        pr.run()
        hist.append((pr.loss_history(), host(pr.field())))
        pr.close()
    assert np.array_equal(hist[0][0], hist[1][0])
    assert np.array_equal(hist[0][1], hist[1][1])


@pytest.mark.parametrize("fused", [False, True], ids=["streams", "fused"])
def test_batched_pairs_match_single_runs(fused):
    """Several registrations advanced together, on their own streams or by
    batched launches, give the results of each run alone (bitwise: the same
    kernel bodies on the same data)."""
    from paper_2404_01249_amd import run_batch
    fixed, moving, _ = make_problem((21, 37, 45), seed=72)
    settings = [dict(eta=0.25), dict(eta=1.0, sigma_warp=0.0), dict(eta=2.0, use_jac=True)]
    ref = []
    for kw in settings:
        pr = new_pair(fixed, moving, **kw)
        pr.set_schedule([2.0, 1.0], [5, 4])
        pr.run()
        ref.append((pr.loss_history(), host(pr.field())))
        pr.close()
    streams = [torch.cuda.Stream() for _ in settings]
    pairs = [Pair(dev(fixed), dev(moving), stream=st, **kw) for st, kw in zip(streams, settings)]
    for pr in pairs:
        pr.set_schedule([2.0, 1.0], [5, 4])
    assert run_batch(pairs, fused=fused) == len(pairs)
    for pr, (loss, field) in zip(pairs, ref):
        if fused:   # the loss partials may be grouped by other chunks
            np.testing.assert_allclose(pr.loss_history(), loss, rtol=1e-6, atol=0)
        else:
            assert np.array_equal(pr.loss_history(), loss)
        got = pr.field()
        pr.stream.synchronize()
        assert np.array_equal(host(got), field)
        pr.close()


UNEVEN_PROBLEMS = [((21, 37, 45), 73), ((40, 48, 56), 74), ((30, 12, 50), 75)]
UNEVEN_CFGS = [(0, dict(eta=0.5), [2.0, 1.0], [5, 4]),
               (1, dict(eta=3.0), [2.0, 1.0], [3, 6]),
               (1, dict(eta=1.0, window=3), [1.0], [7]),
               (2, dict(eta=0.25, use_jac=True), [2.0, 1.0], [4, 2]),
               (0, dict(eta=2.0, sigma_warp=0.0), [4.0, 2.0, 1.0], [2, 3, 2]),
               (1, dict(eta=0.5, window=7, sigma_grad=1.5), [2.0, 1.0], [2, 3]),
               (2, dict(eta=1.0), [1.0], [9]),
               (0, dict(eta=0.25, sigma_grad=6.0, sigma_warp=0.4), [2.0, 1.0], [3, 3])]
_UNEVEN_ORACLE = {}


def uneven_oracle_run(i):
    """The oracle's registration of UNEVEN_CFGS[i] (computed once)."""
    if i not in _UNEVEN_ORACLE:
        k, kw, sc, it = UNEVEN_CFGS[i]
        fixed, moving, _ = make_problem(*UNEVEN_PROBLEMS[k])
        P = O.Params(**kw)
        d_ref, loss_ref, _ = O.register(fixed, moving, sc, it, P)
        _UNEVEN_ORACLE[i] = (d_ref, loss_ref)
    return _UNEVEN_ORACLE[i]


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graphs"])
def test_fused_batch_of_uneven_pairs_matches_single_runs(graphs):
    """Batched launches over pairs that differ in size (brick and march
    launches, 16x32 and 8x32 tiles), window, step size (eta = 3 takes the
    composition with gathers), smoothing, schedule and use_jac, advanced a few
    iterations per call so that the launch tables change as pairs change
    level or finish: every pair gives the field of its run alone, bitwise
    (each voxel's arithmetic does not depend on the launch shape), and the
    oracle's registration to the run tolerances.  With graphs, the first
    iteration of each call runs eagerly and the other two replay the captured
    graph, between the calls' own eager work."""
    from paper_2404_01249_amd import run_batch
    problems = [make_problem(*pr) for pr in UNEVEN_PROBLEMS]
    cfgs = UNEVEN_CFGS
    ref = []
    for k, kw, sc, it in cfgs:
        fixed, moving, _ = problems[k]
        pr = new_pair(fixed, moving, **kw)
        pr.set_schedule(sc, it)
        pr.run()
        ref.append((pr.loss_history(), host(pr.field())))
        pr.close()
    streams = [torch.cuda.Stream() for _ in range(3)]
    pairs = []
    for i, (k, kw, sc, it) in enumerate(cfgs):
        fixed, moving, _ = problems[k]
        pr = Pair(dev(fixed), dev(moving), stream=streams[i % 3] if i % 2 else None, **kw)
        pr.set_schedule(sc, it)
        pairs.append(pr)
    calls, fin = 0, 0
    while fin < len(pairs):
        fin = run_batch(pairs, 3, fused=True, graphs=graphs)
        calls += 1
        assert calls <= 10
    for i, (pr, (loss, field)) in enumerate(zip(pairs, ref)):
        # a batched launch may chunk the march differently, which regroups
        # the loss partials (summed in double, then rounded to float)
        np.testing.assert_allclose(pr.loss_history(), loss, rtol=1e-6, atol=0)
        got = pr.field()
        torch.cuda.synchronize()
        d = host(got)
        assert np.array_equal(d, field), i
        d_ref, loss_ref = uneven_oracle_run(i)
        check_run_against_oracle(pr.loss_history(), d, d_ref, loss_ref, label=f"batch pair {i} {cfgs[i]}")
        pr.close()


def test_step_before_schedule_is_a_state_error():
    fixed, moving, _ = make_problem((8, 9, 10), seed=81)
    pr = new_pair(fixed, moving)
    with pytest.raises(fa.FAError) as e:
        pr.step(1)
    assert e.value.status == fa.FA_ESTATE
    pr.set_schedule([1.0], [2])
    assert pr.step(5) == (2, 1)
    assert pr.step(5) == (0, 1)
    pr.close()


def test_autotune_keeps_state_and_results():
    """The autotuner times launch shapes on scratch outputs: the pair's state
    is unchanged, every chosen shape is a valid one, and the run that follows
    matches an untuned run (to summation order, as bricks may be chosen)."""
    fixed, moving, _ = make_problem((40, 48, 56), seed=91)
    ref = new_pair(fixed, moving)
    ref.set_schedule([2.0, 1.0], [8, 6])
    ref.run()
    ref_loss, ref_d = ref.loss_history(), host(ref.field())
    ref.close()
    try:
        _autotune_checks(fixed, moving, ref_loss, ref_d)
    finally:
        fa.fa_autotune_clear()   # the kept shapes are process-wide


def _autotune_checks(fixed, moving, ref_loss, ref_d):
    pr = new_pair(fixed, moving)
    pr.set_schedule([2.0, 1.0], [8, 6])
    pr.autotune(trials=2)
    d0, m0, v0 = (host(t) for t in pr.state())
    assert not d0.any() and not m0.any() and not v0.any()
    assert pr.progress() == (0, 0, 0)
    for level in (0, 1):
        for kind in range(4):
            ty, tx, zc, brick = pr.tiling(level, kind)
            assert (ty, tx) in ((16, 32), (8, 32), (8, 64), (8, 16)) and zc >= 1
    assert pr.run() == 14
    loss, d = pr.loss_history(), host(pr.field())
    tuned = [[pr.tiling(level, kind) for kind in range(4)] for level in (0, 1)]
    pr.close()
    np.testing.assert_allclose(loss, ref_loss, rtol=1e-4)
    assert np.sqrt(((d - ref_d) ** 2).sum(0)).mean() <= 1e-3
    # later schedules of the same level grids reuse the tuned shapes, until cleared
    q = new_pair(fixed, moving)
    q.set_schedule([2.0, 1.0], [1, 1])
    assert [[q.tiling(level, kind) for kind in range(4)] for level in (0, 1)] == tuned
    fa.fa_autotune_clear()
    q.set_schedule([2.0, 1.0], [1, 1])
    auto = [[q.tiling(level, kind) for kind in range(4)] for level in (0, 1)]
    q.close()
    u = new_pair(fixed, moving)
    u.set_schedule([2.0, 1.0], [1, 1])
    assert [[u.tiling(level, kind) for kind in range(4)] for level in (0, 1)] == auto
    u.close()


def random_configs(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        shape = tuple(int(v) for v in rng.integers(6, 40, 3))
        out.append(dict(shape=shape, window=int(rng.choice([1, 3, 5, 7, 9])),
                        sigma_grad=float(rng.choice([0.0, 0.5, 1.0, 1.5])),
                        sigma_warp=float(rng.choice([0.0, 0.5, 1.0])),
                        eta=float(rng.choice([0.25, 1.0, 3.0])), use_jac=bool(rng.integers(0, 2)),
                        seed=int(rng.integers(0, 10000))))
    return out


@pytest.mark.parametrize("cfg", random_configs(12, 2024), ids=lambda c: "x".join(map(str, c["shape"])) +
                         f"-w{c['window']}-g{c['sigma_grad']}-s{c['sigma_warp']}-e{c['eta']}-j{int(c['use_jac'])}")
def test_random_configurations_match_oracle(cfg):
    """Seeded random shapes, windows, Gaussian widths, step sizes (eta = 3
    takes the composition with gathers) and use_jac: a two-level run of 3 + 2
    iterations against the oracle (loss history and final field)."""
    fixed, moving, _ = make_problem(cfg["shape"], seed=cfg["seed"])
    kw = {k: cfg[k] for k in ("window", "sigma_grad", "sigma_warp", "eta", "use_jac")}
    scales, iters = [2.0, 1.0], [3, 2]
    if min(cfg["shape"]) < 8:
        scales, iters = [1.0], [4]
    pr = new_pair(fixed, moving, **kw)
    pr.set_schedule(scales, iters)
    assert pr.run() == sum(iters)
    loss = pr.loss_history().astype(np.float64)
    d = host(pr.field())
    pr.close()
    P = O.Params(eta=cfg["eta"], sigma_grad=cfg["sigma_grad"], sigma_warp=cfg["sigma_warp"], window=cfg["window"],
                 use_jac=cfg["use_jac"])
    d_ref, loss_ref, _ = O.register(fixed, moving, scales, iters, P)
    rel = np.abs(loss - np.asarray(loss_ref)) / np.maximum(np.abs(loss_ref), 1e-12)
    epe = np.sqrt(((d - d_ref) ** 2).sum(0))
    q = float(np.quantile(epe, 0.999))
    print(f"{cfg}: loss rel max {rel.max():.2e}, endpoint diff mean {epe.mean():.2e} "
          f"99.9% {q:.2e} max {epe.max():.2e}")
    assert rel[0] <= 1e-5 and rel.max() <= 1e-3
    # The position derivative jumps where a sample crosses a cell boundary
    # (the cell is the floor of the position).  A sample within fp32 rounding
    # of an integer can take the other cell than in the oracle's fp64 state,
    # and Adam's per-voxel normalisation turns that into a full-size step
    # difference at that voxel: large steps (eta = 3) with no warp smoothing
    # show it at a voxel or two.  The mean and nearly every voxel stay close.
    assert epe.mean() <= 1e-3 and q <= 0.05
