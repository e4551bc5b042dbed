"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the public headers declare, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_01249_amd import fa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for h in sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(fa_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fa.LIB_PATH):
        pytest.fail("HIP library not built (python -m paper_2404_01249_amd.build)")
    return fa.load_library()


def test_library_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "fa_pair_create" in names and "fa_pair_step" in names and "fa_pair_eval_gradient" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(fa.SIGNATURES)


def test_params_default(lib):
    p = fa.fa_params_default()
    assert p.cc_window == 5 and p.use_jac == 0
    assert p.eta == pytest.approx(0.5) and p.adam_beta2 == pytest.approx(0.999)


def _create_raw(lib, params, shape=(8, 8, 8), ptrs=(1, 2)):
    h = ctypes.c_void_p()
    st = lib.fa_pair_create(ptrs[0], ptrs[1], fa.fa_shape(*shape), ctypes.byref(params), None, ctypes.byref(h))
    return st, h.value


@pytest.mark.parametrize("field,value", [("cc_window", 4), ("cc_window", 11), ("cc_window", 0),
                                         ("eta", 0.0), ("eta", -1.0), ("use_jac", 2),
                                         ("sigma_grad", 8.5), ("sigma_warp", 100.0), ("adam_beta1", 1.0),
                                         ("cc_eps", -1.0)])
def test_invalid_params_rejected_before_device_work(lib, field, value):
    p = fa.fa_params_default()
    setattr(p, field, value)
    st, h = _create_raw(lib, p)
    assert st == fa.FA_EINVAL and h is None
    assert len(fa.fa_last_error()) > 0


@pytest.mark.parametrize("shape", [(1, 8, 8), (8, 0, 8), (2048, 2048, 256)])
def test_invalid_shapes_rejected(lib, shape):
    st, h = _create_raw(lib, fa.fa_params_default(), shape=shape)
    assert st == fa.FA_ESHAPE and h is None


def test_null_pointers_rejected(lib):
    st, h = _create_raw(lib, fa.fa_params_default(), ptrs=(None, None))
    assert st == fa.FA_EINVAL
    assert lib.fa_pair_step(None, 1, None, None) == fa.FA_EINVAL
    assert lib.fa_pair_set_schedule(None, 1, None, None) == fa.FA_EINVAL
    lib.fa_pair_destroy(None)


@pytest.mark.parametrize("name", ["fa_batch_step", "fa_batch_step_fused"])
def test_batch_step_rejects_bad_arguments(lib, name):
    fn = getattr(lib, name)
    fin = ctypes.c_int(7)
    assert fn(None, 0, 1, ctypes.byref(fin)) == fa.FA_OK and fin.value == 0
    assert fn(None, 2, 1, None) == fa.FA_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert fn(arr, 1, 1, None) == fa.FA_EINVAL
    assert fn(arr, 1, -1, None) == fa.FA_EINVAL


def test_plan_tiling_single_volumes():
    """The automatic march chunks of one registration's launches: the
    longest chunk that keeps the launch within the resident workgroups
    (512 for the gradient kernel, 1024 for the sigma_grad smoothing)."""
    assert fa.fa_plan_tiling(0, [(160, 192, 224)], 8, False) == ([27], [504])
    assert fa.fa_plan_tiling(0, [(80, 96, 112)], 8, False) == ([4], [480])
    assert fa.fa_plan_tiling(1, [(160, 192, 224)], 6, False) == ([14], [1008])
    # smoothing chunks are at least 4 planes (their halo is 2R planes)
    assert fa.fa_plan_tiling(1, [(40, 48, 56)], 6, False) == ([4], [60])


def test_plan_tiling_batched_chunks_cover_every_volume():
    rng = np.random.default_rng(5)
    for trial in range(60):
        kind = int(rng.integers(0, 4))
        n = int(rng.integers(1, 9))
        shapes = [tuple(int(v) for v in rng.integers(2, 260, 3)) for _ in range(n)]
        halo = int(rng.integers(0, 13))
        zs, bs = fa.fa_plan_tiling(kind, shapes, halo, False)
        zb, bb = fa.fa_plan_tiling(kind, shapes, halo, True)
        if n == 1:
            assert (zb, bb) == (zs, bs)   # a launch of one keeps its own chunk
        for (n0, n1, n2), z, b in zip(shapes, zb, bb):
            ty = 16 if n1 >= 16 else 8
            tiles = -(-n1 // ty) * -(-n2 // 32)
            chunks = -(-n0 // z)
            assert 1 <= z <= n0
            assert (chunks - 1) * z < n0 <= chunks * z
            assert b == tiles * chunks


def test_plan_tiling_batch_lengthens_chunks():
    """Four 80x96x112 volumes share the 512 resident gradient workgroups:
    16-plane chunks (a third of the halo recomputation of 4-plane ones) fill
    them in one round."""
    zc, nb = fa.fa_plan_tiling(0, [(80, 96, 112)] * 4, 8, True)
    assert zc == [16] * 4 and nb == [120] * 4
    zc, nb = fa.fa_plan_tiling(0, [(160, 192, 224)] * 4, 8, True)
    assert zc == [54] * 4 and sum(nb) == 1008


def test_plan_tiling_rejects_bad_arguments(lib):
    arr = (fa.fa_shape * 1)(fa.fa_shape(10, 10, 10))
    assert lib.fa_plan_tiling(4, 1, arr, 0, 0, None, None) == fa.FA_EINVAL
    assert lib.fa_plan_tiling(0, 0, arr, 0, 0, None, None) == fa.FA_EINVAL
    assert lib.fa_plan_tiling(0, 1, None, 0, 0, None, None) == fa.FA_EINVAL
    assert lib.fa_plan_tiling(0, 1, arr, -1, 0, None, None) == fa.FA_EINVAL
    bad = (fa.fa_shape * 1)(fa.fa_shape(1, 10, 10))
    assert lib.fa_plan_tiling(0, 1, bad, 0, 0, None, None) == fa.FA_ESHAPE


def test_inverse_rejects_bad_arguments_before_any_device_work(lib):
    p = fa.fa_params_default()
    shp = fa.fa_shape(8, 9, 10)
    h = ctypes.c_void_p(0)
    assert lib.fa_inverse_create(None, shp, ctypes.byref(p), None, ctypes.byref(h)) == fa.FA_EINVAL
    assert lib.fa_inverse_create(ctypes.c_void_p(16), shp, ctypes.byref(p), None, None) == fa.FA_EINVAL
    assert lib.fa_inverse_create(ctypes.c_void_p(16), fa.fa_shape(1, 9, 10), ctypes.byref(p), None,
                                 ctypes.byref(h)) == fa.FA_ESHAPE
    bad = fa.fa_params_default()
    bad.eta = -1.0
    assert lib.fa_inverse_create(ctypes.c_void_p(16), shp, ctypes.byref(bad), None, ctypes.byref(h)) == fa.FA_EINVAL
    assert lib.fa_inverse_set_schedule(None, 1, None, None) == fa.FA_EINVAL
    assert lib.fa_inverse_step(None, 1, None, None) == fa.FA_EINVAL
    assert lib.fa_inverse_get_field(None, None, None, None) == fa.FA_EINVAL
    assert lib.fa_inverse_get_loss(None, None, 0, None) == fa.FA_EINVAL
    assert lib.fa_inverse_eval_gradient(None, None, None) == fa.FA_EINVAL
    assert lib.fa_inverse_set_splat(None, 0) == fa.FA_EINVAL
    lib.fa_inverse_destroy(None)


def test_symmetric_rejects_bad_arguments_before_any_device_work(lib):
    p = fa.fa_params_default()
    shp = fa.fa_shape(8, 9, 10)
    h = ctypes.c_void_p(0)
    assert lib.fa_sym_create(None, None, shp, ctypes.byref(p), None, ctypes.byref(h)) == fa.FA_EINVAL
    assert lib.fa_sym_create(ctypes.c_void_p(16), ctypes.c_void_p(16), shp, ctypes.byref(p), None, None) == fa.FA_EINVAL
    assert lib.fa_sym_set_schedule(None, 1, None, None) == fa.FA_EINVAL
    assert lib.fa_sym_step(None, 1, None, None) == fa.FA_EINVAL
    assert lib.fa_sym_get_halfway(None, None, None, None, None) == fa.FA_EINVAL
    assert lib.fa_sym_get_loss(None, None, 0, None) == fa.FA_EINVAL
    assert lib.fa_sym_finish(None, ctypes.byref(p), 1, None, None, None, None) == fa.FA_EINVAL
    lib.fa_sym_destroy(None)


def test_autotune_rejects_bad_arguments(lib):
    assert lib.fa_pair_autotune(None, 5) == fa.FA_EINVAL
    assert lib.fa_pair_get_tiling(None, 0, 0, None, None, None, None) == fa.FA_EINVAL


def test_compose_fields_rejects_bad_arguments(lib):
    shp = fa.fa_shape(4, 5, 6)
    p = ctypes.c_void_p
    assert lib.fa_compose_fields(None, p(32), shp, p(64), None) == fa.FA_EINVAL
    assert lib.fa_compose_fields(p(16), p(32), shp, p(32), None) == fa.FA_EINVAL   # out aliases d
    assert lib.fa_compose_fields(p(16), p(32), fa.fa_shape(1, 5, 6), p(64), None) == fa.FA_ESHAPE


def test_noalloc_lncc_rejects_bad_arguments_before_device_work(lib):
    fn = lib.fa_lncc_eval_noalloc
    ok = fa.fa_shape(8, 8, 8)
    # a volume whose padded copy exceeds the fixed scratch array (204^3 floats > 32 MiB)
    assert fn(fa.fa_shape(200, 200, 200), 5, 1e-5, 1, 2, 3, 4, 5, None, None) == fa.FA_EINVAL
    assert "too large" in fa.fa_last_error()
    assert fn(ok, 4, 1e-5, 1, 2, 3, 4, 5, None, None) == fa.FA_EINVAL          # even window
    assert fn(ok, 5, -1.0, 1, 2, 3, 4, 5, None, None) == fa.FA_EINVAL         # negative eps
    assert fn(ok, 5, 1e-5, None, 2, 3, 4, 5, None, None) == fa.FA_EINVAL      # null input
    assert fn(ok, 5, 1e-5, 1, 2, 3, None, None, None, None) == fa.FA_EINVAL   # no output
    assert fn(fa.fa_shape(1, 8, 8), 5, 1e-5, 1, 2, 3, 4, 5, None, None) == fa.FA_ESHAPE


@pytest.mark.parametrize("sigma", [2.5, 6.0, 8.0])
def test_wide_gaussians_pass_validation(lib, sigma):
    """Radii ceil(3 sigma) up to 24 (sigma <= 8 voxels) pass parameter
    validation: creation gets past it (and, without a GPU, stops at the first
    device call instead)."""
    p = fa.fa_params_default()
    p.sigma_grad = sigma
    p.sigma_warp = sigma
    st, h = _create_raw(lib, p)
    assert st != fa.FA_EINVAL, fa.fa_last_error()
    if h is not None:
        lib.fa_pair_destroy(h)
