"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the public headers declare, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

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
                                         ("sigma_grad", 2.5), ("adam_beta1", 1.0), ("cc_eps", -1.0)])
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


def test_batch_step_rejects_bad_arguments(lib):
    fin = ctypes.c_int(7)
    assert lib.fa_batch_step(None, 0, 1, ctypes.byref(fin)) == fa.FA_OK and fin.value == 0
    assert lib.fa_batch_step(None, 2, 1, None) == fa.FA_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.fa_batch_step(arr, 1, 1, None) == fa.FA_EINVAL
    assert lib.fa_batch_step(arr, 1, -1, None) == fa.FA_EINVAL
