"""ctypes binding of the C ABI in include/fa.h, include/fa_inspect.h,
include/fa_batch.h, include/fa_lncc.h and include/fa_eval.h.

Each function has the name of the C entry point it wraps and only marshals
arguments: torch tensors become device pointers, the stream becomes its HIP
handle, and a non-OK status raises :class:`FAError` with the library's
message.  All computation happens in the HIP library; there is no fallback,
and loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfa_mi355x.so")

FA_OK, FA_EINVAL, FA_ESHAPE, FA_ENOMEM, FA_EHIP, FA_ESTATE = 0, -1, -2, -3, -4, -5
_STATUS_NAMES = {0: "FA_OK", -1: "FA_EINVAL", -2: "FA_ESHAPE", -3: "FA_ENOMEM", -4: "FA_EHIP", -5: "FA_ESTATE"}


class FAError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class fa_shape(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int), ("n1", ctypes.c_int), ("n2", ctypes.c_int)]


class fa_params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_float), ("sigma_grad", ctypes.c_float), ("sigma_warp", ctypes.c_float),
        ("cc_window", ctypes.c_int), ("cc_eps", ctypes.c_float), ("adam_beta1", ctypes.c_float),
        ("adam_beta2", ctypes.c_float), ("adam_eps", ctypes.c_float), ("use_jac", ctypes.c_int),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_IP = ctypes.POINTER(ctypes.c_int)
_FP = ctypes.POINTER(ctypes.c_float)
_I64 = ctypes.c_int64
_I64P = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "fa_params_default": (_I, [ctypes.POINTER(fa_params)]),
    "fa_pair_create": (_I, [_P, _P, fa_shape, ctypes.POINTER(fa_params), _P, ctypes.POINTER(_P)]),
    "fa_pair_set_schedule": (_I, [_P, _I, _FP, _IP]),
    "fa_pair_step": (_I, [_P, _I, _IP, _IP]),
    "fa_pair_get_loss": (_I, [_P, _FP, _I, _IP]),
    "fa_pair_get_field": (_I, [_P, _P, _I, _IP, ctypes.POINTER(fa_shape)]),
    "fa_pair_get_warped": (_I, [_P, _P]),
    "fa_pair_destroy": (None, [_P]),
    "fa_last_error": (ctypes.c_char_p, []),
    "fa_pair_get_progress": (_I, [_P, _IP, _IP, _IP]),
    "fa_pair_set_state": (_I, [_P, _P, _P, _P, _I]),
    "fa_pair_get_state": (_I, [_P, _P, _P, _P]),
    "fa_pair_eval_gradient": (_I, [_P, _P, _FP]),
    "fa_pair_get_direction": (_I, [_P, _P]),
    "fa_pair_get_step_norm": (_I, [_P, _FP]),
    "fa_pair_get_level_image": (_I, [_P, _I, _I, _P, ctypes.POINTER(fa_shape)]),
    "fa_pair_profile": (_I, [_P, _I]),
    "fa_pair_set_tuning": (_I, [_P, _I, _I, _I, _I, _I]),
    "fa_pair_get_profile": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_double), _IP]),
    "fa_batch_step": (_I, [ctypes.POINTER(_P), _I, _I, _IP]),
    "fa_batch_step_fused": (_I, [ctypes.POINTER(_P), _I, _I, _IP]),
    "fa_batch_use_graphs": (None, [_I]),
    "fa_plan_tiling": (_I, [_I, _I, ctypes.POINTER(fa_shape), _I, _I, _IP, _IP]),
    "fa_pair_autotune": (_I, [_P, _I]),
    "fa_pair_get_tiling": (_I, [_P, _I, _I, _IP, _IP, _IP, _IP]),
    "fa_autotune_clear": (None, []),
    "fa_inverse_create": (_I, [_P, fa_shape, ctypes.POINTER(fa_params), _P, ctypes.POINTER(_P)]),
    "fa_inverse_set_schedule": (_I, [_P, _I, _FP, _IP]),
    "fa_inverse_step": (_I, [_P, _I, _IP, _IP]),
    "fa_inverse_get_field": (_I, [_P, _P, _IP, ctypes.POINTER(fa_shape)]),
    "fa_inverse_get_loss": (_I, [_P, _FP, _I, _IP]),
    "fa_inverse_eval_gradient": (_I, [_P, _P, _FP]),
    "fa_inverse_destroy": (None, [_P]),
    "fa_inverse_set_splat": (_I, [_P, _I]),
    "fa_sym_create": (_I, [_P, _P, fa_shape, ctypes.POINTER(fa_params), _P, ctypes.POINTER(_P)]),
    "fa_sym_set_schedule": (_I, [_P, _I, _FP, _IP]),
    "fa_sym_step": (_I, [_P, _I, _IP, _IP]),
    "fa_sym_get_halfway": (_I, [_P, _P, _P, _IP, ctypes.POINTER(fa_shape)]),
    "fa_sym_get_loss": (_I, [_P, _FP, _I, _IP]),
    "fa_sym_finish": (_I, [_P, ctypes.POINTER(fa_params), _I, _FP, _IP, _P, _FP]),
    "fa_sym_destroy": (None, [_P]),
    "fa_lncc_create": (_I, [fa_shape, _I, ctypes.c_float, _P, ctypes.POINTER(_P)]),
    "fa_lncc_eval": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "fa_lncc_destroy": (None, [_P]),
    "fa_lncc_eval_noalloc": (_I, [fa_shape, _I, ctypes.c_float, _P, _P, _P, _P, _P, _P, _P]),
    "fa_warp_labels": (_I, [_P, _P, fa_shape, _P, _P]),
    "fa_label_overlap": (_I, [_P, _P, _I64, _I, _I64P, _P]),
    "fa_jacobian_det": (_I, [_P, fa_shape, _P, _I64P, _I64P, _P]),
    "fa_compose_fields": (_I, [_P, _P, fa_shape, _P, _P]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_2404_01249_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != FA_OK:
        raise FAError(status, load_library().fa_last_error().decode(errors="replace"))


def _ptr(t) -> int | None:
    """Device pointer of a float32 contiguous GPU tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype.itemsize != 4 or not t.is_floating_point():
        raise ValueError("tensor must be float32")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _ptr_typed(t, dtype_name: str) -> int | None:
    """Device pointer of a contiguous GPU tensor of the given torch dtype (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"tensor must be {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---- one wrapper per entry point, same names --------------------------------

def fa_params_default() -> fa_params:
    p = fa_params()
    _check(load_library().fa_params_default(ctypes.byref(p)))
    return p


def fa_pair_create(fixed, moving, params: fa_params, stream=None) -> int:
    if fixed.shape != moving.shape or fixed.dim() != 3:
        raise ValueError("fixed and moving must be 3-D volumes of the same shape")
    shape = fa_shape(*[int(s) for s in fixed.shape])
    h = _P()
    _check(load_library().fa_pair_create(_ptr(fixed), _ptr(moving), shape, ctypes.byref(params),
                                         _stream_handle(stream), ctypes.byref(h)))
    return h.value


def fa_pair_set_schedule(pair: int, scales, iters):
    scales = np.ascontiguousarray(scales, dtype=np.float32)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    if scales.shape != iters.shape or scales.ndim != 1:
        raise ValueError("scales and iters must be 1-D of equal length")
    _check(load_library().fa_pair_set_schedule(pair, len(scales), scales.ctypes.data_as(_FP),
                                               iters.ctypes.data_as(_IP)))


def fa_pair_step(pair: int, max_iters: int) -> tuple[int, int]:
    done, fin = ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().fa_pair_step(pair, int(max_iters), ctypes.byref(done), ctypes.byref(fin)))
    return done.value, fin.value


def fa_pair_get_loss(pair: int, capacity: int) -> np.ndarray:
    out = np.zeros(max(int(capacity), 0), dtype=np.float32)
    n = ctypes.c_int(0)
    _check(load_library().fa_pair_get_loss(pair, out.ctypes.data_as(_FP), len(out), ctypes.byref(n)))
    return out[: n.value]


def fa_pair_get_field(pair: int, dev_out=None, layout: int = 0) -> tuple[int, tuple]:
    lvl, shp = ctypes.c_int(0), fa_shape()
    _check(load_library().fa_pair_get_field(pair, _ptr(dev_out), int(layout), ctypes.byref(lvl),
                                            ctypes.byref(shp)))
    return lvl.value, (shp.n0, shp.n1, shp.n2)


def fa_pair_get_warped(pair: int, dev_out):
    _check(load_library().fa_pair_get_warped(pair, _ptr(dev_out)))


def fa_pair_destroy(pair: int):
    if pair:
        load_library().fa_pair_destroy(pair)


def fa_last_error() -> str:
    return load_library().fa_last_error().decode(errors="replace")


def fa_pair_get_progress(pair: int) -> tuple[int, int, int]:
    a, b, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().fa_pair_get_progress(pair, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def fa_pair_set_state(pair: int, d=None, m=None, v=None, t_done: int = 0):
    _check(load_library().fa_pair_set_state(pair, _ptr(d), _ptr(m), _ptr(v), int(t_done)))


def fa_pair_get_state(pair: int, d=None, m=None, v=None):
    _check(load_library().fa_pair_get_state(pair, _ptr(d), _ptr(m), _ptr(v)))


def fa_pair_eval_gradient(pair: int, g_dev=None) -> float:
    loss = ctypes.c_float(0.0)
    _check(load_library().fa_pair_eval_gradient(pair, _ptr(g_dev), ctypes.byref(loss)))
    return float(loss.value)


def fa_pair_get_direction(pair: int, dev_out):
    _check(load_library().fa_pair_get_direction(pair, _ptr(dev_out)))


def fa_pair_get_step_norm(pair: int) -> float:
    m = ctypes.c_float(0.0)
    _check(load_library().fa_pair_get_step_norm(pair, ctypes.byref(m)))
    return float(m.value)


def fa_pair_get_level_image(pair: int, level: int, which: int, dev_out=None) -> tuple:
    shp = fa_shape()
    _check(load_library().fa_pair_get_level_image(pair, int(level), int(which), _ptr(dev_out),
                                                  ctypes.byref(shp)))
    return (shp.n0, shp.n1, shp.n2)


def fa_pair_profile(pair: int, enable: bool):
    _check(load_library().fa_pair_profile(pair, 1 if enable else 0))


def fa_pair_get_profile(pair: int, level: int, kind: int) -> tuple[float, int]:
    ms, n = ctypes.c_double(0.0), ctypes.c_int(0)
    _check(load_library().fa_pair_get_profile(pair, int(level), int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), n.value


def fa_pair_set_tuning(pair: int, kind: int, ty: int = 0, tx: int = 0, zc: int = 0, variant: int = 0):
    _check(load_library().fa_pair_set_tuning(pair, int(kind), int(ty), int(tx), int(zc), int(variant)))


# ---- include/fa_lncc.h --------------------------------------------------------

def fa_lncc_create(shape, window: int = 5, cc_eps: float = 1e-5, stream=None) -> int:
    h = _P()
    _check(load_library().fa_lncc_create(fa_shape(*[int(x) for x in shape]), int(window), float(cc_eps),
                                         _stream_handle(stream), ctypes.byref(h)))
    return h.value


def fa_lncc_eval(h: int, fixed, moving, d, loss_dev=None, grad_dev=None, grad_scale_dev=None):
    _check(load_library().fa_lncc_eval(h, _ptr(fixed), _ptr(moving), _ptr(d), _ptr(loss_dev), _ptr(grad_dev),
                                       _ptr(grad_scale_dev)))


def fa_lncc_destroy(h: int):
    if h:
        load_library().fa_lncc_destroy(h)


def fa_lncc_eval_noalloc(shape, window: int, cc_eps: float, fixed, moving, d, loss_dev=None, grad_dev=None,
                         grad_scale_dev=None, stream=None):
    _check(load_library().fa_lncc_eval_noalloc(fa_shape(*[int(x) for x in shape]), int(window), float(cc_eps),
                                               _ptr(fixed), _ptr(moving), _ptr(d), _ptr(loss_dev), _ptr(grad_dev),
                                               _ptr(grad_scale_dev), _stream_handle(stream)))


# ---- include/fa_eval.h --------------------------------------------------------

def fa_warp_labels(labels, d, out, stream=None):
    shape = fa_shape(*[int(x) for x in labels.shape])
    _check(load_library().fa_warp_labels(_ptr_typed(labels, "int8"), _ptr(d), shape, _ptr_typed(out, "int8"),
                                         _stream_handle(stream)))


def fa_label_overlap(a, b, n_classes: int, stream=None) -> np.ndarray:
    if a.numel() != b.numel():
        raise ValueError("a and b must have the same number of voxels")
    counts = np.zeros(3 * int(n_classes), dtype=np.int64)
    _check(load_library().fa_label_overlap(_ptr_typed(a, "int8"), _ptr_typed(b, "int8"), int(a.numel()),
                                           int(n_classes), counts.ctypes.data_as(_I64P), _stream_handle(stream)))
    return counts.reshape(int(n_classes), 3)


def fa_jacobian_det(d, det_out=None, count: bool = True, stream=None) -> tuple[int, int]:
    if d.dim() != 4 or d.shape[0] != 3:
        raise ValueError("d must be (3, n0, n1, n2)")
    shape = fa_shape(*[int(x) for x in d.shape[1:]])
    nonpos, interior = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().fa_jacobian_det(_ptr(d), shape, _ptr_typed(det_out, "float64"),
                                          ctypes.byref(nonpos) if count else None, ctypes.byref(interior),
                                          _stream_handle(stream)))
    return nonpos.value, interior.value


# ---- include/fa_batch.h -------------------------------------------------------

def fa_batch_step(pairs, max_iters: int) -> int:
    arr = (_P * len(pairs))(*pairs)
    fin = ctypes.c_int(0)
    _check(load_library().fa_batch_step(arr, len(pairs), int(max_iters), ctypes.byref(fin)))
    return fin.value


def fa_pair_autotune(pair: int, trials: int = 5):
    _check(load_library().fa_pair_autotune(pair, int(trials)))


def fa_autotune_clear():
    load_library().fa_autotune_clear()


def fa_pair_get_tiling(pair: int, level: int, kind: int) -> tuple[int, int, int, bool]:
    ty, tx, zc, br = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().fa_pair_get_tiling(pair, int(level), int(kind), ctypes.byref(ty), ctypes.byref(tx),
                                             ctypes.byref(zc), ctypes.byref(br)))
    return ty.value, tx.value, zc.value, bool(br.value)


def fa_plan_tiling(kind: int, shapes, halo: int, batched: bool):
    """Automatic march chunks (planes per workgroup) and workgroup counts for
    volumes of the given shapes: each alone, or in one batched launch."""
    n = len(shapes)
    arr = (fa_shape * n)(*[fa_shape(*map(int, s)) for s in shapes])
    zc = (ctypes.c_int * n)()
    nb = (ctypes.c_int * n)()
    _check(load_library().fa_plan_tiling(int(kind), n, arr, int(halo), int(bool(batched)), zc, nb))
    return list(zc), list(nb)


def fa_inverse_create(d, params: fa_params, stream=None) -> int:
    if d.dim() != 4 or d.shape[0] != 3:
        raise ValueError("d must be a (3, n0, n1, n2) displacement")
    shape = fa_shape(*[int(s) for s in d.shape[1:]])
    h = _P()
    _check(load_library().fa_inverse_create(_ptr(d), shape, ctypes.byref(params), _stream_handle(stream),
                                            ctypes.byref(h)))
    return h.value


def fa_inverse_set_schedule(h: int, scales, iters):
    scales = np.ascontiguousarray(scales, dtype=np.float32)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    if scales.shape != iters.shape or scales.ndim != 1:
        raise ValueError("scales and iters must be 1-D of equal length")
    _check(load_library().fa_inverse_set_schedule(h, len(scales), scales.ctypes.data_as(_FP),
                                                  iters.ctypes.data_as(_IP)))


def fa_inverse_step(h: int, max_iters: int) -> tuple[int, int]:
    done, fin = ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().fa_inverse_step(h, int(max_iters), ctypes.byref(done), ctypes.byref(fin)))
    return done.value, fin.value


def fa_inverse_get_field(h: int, dev_out=None) -> tuple[int, tuple]:
    lvl, shp = ctypes.c_int(0), fa_shape()
    _check(load_library().fa_inverse_get_field(h, _ptr(dev_out), ctypes.byref(lvl), ctypes.byref(shp)))
    return lvl.value, (shp.n0, shp.n1, shp.n2)


def fa_inverse_get_loss(h: int, capacity: int) -> np.ndarray:
    out = np.zeros(max(int(capacity), 0), dtype=np.float32)
    n = ctypes.c_int(0)
    _check(load_library().fa_inverse_get_loss(h, out.ctypes.data_as(_FP), len(out), ctypes.byref(n)))
    return out[: n.value]


def fa_inverse_eval_gradient(h: int, g_dev) -> float:
    loss = ctypes.c_float(0.0)
    _check(load_library().fa_inverse_eval_gradient(h, _ptr(g_dev), ctypes.byref(loss)))
    return loss.value


def fa_inverse_set_splat(h: int, direct: bool):
    _check(load_library().fa_inverse_set_splat(h, int(bool(direct))))


def fa_inverse_destroy(h: int):
    if h:
        load_library().fa_inverse_destroy(h)


def fa_sym_create(fixed, moving, params: fa_params, stream=None) -> int:
    if fixed.shape != moving.shape or fixed.dim() != 3:
        raise ValueError("fixed and moving must be 3-D volumes of the same shape")
    shape = fa_shape(*[int(s) for s in fixed.shape])
    h = _P()
    _check(load_library().fa_sym_create(_ptr(fixed), _ptr(moving), shape, ctypes.byref(params),
                                        _stream_handle(stream), ctypes.byref(h)))
    return h.value


def fa_sym_set_schedule(h: int, scales, iters):
    scales = np.ascontiguousarray(scales, dtype=np.float32)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    if scales.shape != iters.shape or scales.ndim != 1:
        raise ValueError("scales and iters must be 1-D of equal length")
    _check(load_library().fa_sym_set_schedule(h, len(scales), scales.ctypes.data_as(_FP), iters.ctypes.data_as(_IP)))


def fa_sym_step(h: int, max_iters: int) -> tuple[int, int]:
    done, fin = ctypes.c_int(0), ctypes.c_int(0)
    _check(load_library().fa_sym_step(h, int(max_iters), ctypes.byref(done), ctypes.byref(fin)))
    return done.value, fin.value


def fa_sym_get_halfway(h: int, dF=None, dM=None) -> tuple[int, tuple]:
    lvl, shp = ctypes.c_int(0), fa_shape()
    _check(load_library().fa_sym_get_halfway(h, _ptr(dF), _ptr(dM), ctypes.byref(lvl), ctypes.byref(shp)))
    return lvl.value, (shp.n0, shp.n1, shp.n2)


def fa_sym_get_loss(h: int, capacity: int) -> np.ndarray:
    out = np.zeros(max(int(capacity), 0), dtype=np.float32)
    n = ctypes.c_int(0)
    _check(load_library().fa_sym_get_loss(h, out.ctypes.data_as(_FP), len(out), ctypes.byref(n)))
    return out[: n.value]


def fa_sym_finish(h: int, inv_params: fa_params, scales, iters, d_out) -> float:
    scales = np.ascontiguousarray(scales, dtype=np.float32)
    iters = np.ascontiguousarray(iters, dtype=np.int32)
    if scales.shape != iters.shape or scales.ndim != 1:
        raise ValueError("scales and iters must be 1-D of equal length")
    cost = ctypes.c_float(0.0)
    _check(load_library().fa_sym_finish(h, ctypes.byref(inv_params), len(scales), scales.ctypes.data_as(_FP),
                                        iters.ctypes.data_as(_IP), _ptr(d_out), ctypes.byref(cost)))
    return cost.value


def fa_sym_destroy(h: int):
    if h:
        load_library().fa_sym_destroy(h)


def fa_batch_use_graphs(enable: bool):
    load_library().fa_batch_use_graphs(int(bool(enable)))


def fa_batch_step_fused(pairs, max_iters: int) -> int:
    arr = (_P * len(pairs))(*pairs)
    fin = ctypes.c_int(0)
    _check(load_library().fa_batch_step_fused(arr, len(pairs), int(max_iters), ctypes.byref(fin)))
    return fin.value


def fa_compose_fields(u, d, out, stream=None):
    if u.shape != d.shape or u.shape != out.shape or u.dim() != 4 or u.shape[0] != 3:
        raise ValueError("u, d and out must be (3, n0, n1, n2) fields of one shape")
    shape = fa_shape(*[int(s) for s in u.shape[1:]])
    _check(load_library().fa_compose_fields(_ptr(u), _ptr(d), shape, _ptr(out), _stream_handle(stream)))
