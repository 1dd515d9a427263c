"""ctypes binding of librwgt.so (include/rwgt.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Device arrays are
torch tensors on the GPU (their data pointers are passed); param_sets is a
host array.  The library must have been built (``python -m
paper_2510_05100_amd.build``); there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# RWGT_LIBRARY=check selects the bounds-checked build (librwgt_check.so).
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "librwgt_check.so" if os.environ.get("RWGT_LIBRARY") == "check" else "librwgt.so")

RWGT_FP64, RWGT_MIXED_FP16, RWGT_MIXED_BF16 = 0, 1, 2
ERRORS = {-1: "RWGT_EINVAL", -2: "RWGT_EPROCESS", -3: "RWGT_ECARD", -4: "RWGT_EDEVICE",
          -5: "RWGT_ENOMEM", -6: "RWGT_EPARAM"}

# symbol name -> (restype, argtypes), exactly as declared in include/rwgt.h
SIGNATURES = {
    "rwgt_create": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_destroy": (None, [ctypes.c_void_p]),
    "rwgt_param_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_char_p)]),
    "rwgt_original_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rwgt_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rwgt_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p]),
    "rwgt_eval_alphas": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_int32, ctypes.c_void_p]),
    "rwgt_eval_factored": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p]),
    "rwgt_me2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p]),
    "rwgt_nonfinite": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "rwgt_create_error": (ctypes.c_char_p, []),
    "rwgt_process_info": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "rwgt_flops": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rwgt_flops_executed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "rwgt_bounds_check": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]),
    "rwgt_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "rwgt_kernel_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float)]),
}

class Segment(ctypes.Structure):
    """rwgt_segment of include/rwgt.h."""
    _fields_ = [("ctx", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nevt", ctypes.c_int64),
                ("momenta", ctypes.c_void_p), ("weights_in", ctypes.c_void_p),
                ("params", ctypes.POINTER(ctypes.c_double)), ("weights_out", ctypes.c_void_p)]


SIGNATURES.update({
    "rwgt_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_batch_destroy": (None, [ctypes.c_void_p]),
    "rwgt_batch_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rwgt_batch_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Segment), ctypes.c_int32]),
    "rwgt_batch_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "rwgt_batch_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32]),
    "rwgt_batch_get_schedule": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "rwgt_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Segment), ctypes.c_int32, ctypes.c_int32]),
    "rwgt_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
})

SIGNATURES.update({
    "rwgt_mlp_create": (ctypes.c_int, [ctypes.c_int32] * 5 + [ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_mlp_destroy": (None, [ctypes.c_void_p]),
    "rwgt_mlp_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rwgt_mlp_num_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "rwgt_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "rwgt_mlp_get_grads": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "rwgt_mlp_set_normalisation": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                  ctypes.POINTER(ctypes.c_float)]),
    "rwgt_mlp_set_training": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_float] * 4),
    "rwgt_mlp_set_calibration": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float]),
    "rwgt_mlp_input_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_mlp_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_void_p]),
    "rwgt_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "rwgt_mlp_set_features": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_int32] * 4 + [ctypes.c_double] * 2),
    "rwgt_mlp_set_target_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float]),
    "rwgt_mlp_fit_normalisation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "rwgt_mlp_fit_target_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "rwgt_mlp_get_normalisation": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_float)] * 3),
    "rwgt_mlp_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "rwgt_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_float, ctypes.c_void_p]),
    "rwgt_mlp_targets": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p]),
    "rwgt_mlp_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "rwgt_eval_cards": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "rwgt_sur_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int64)]),
})

SIGNATURES.update({
    "rwgt_lhe_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_lhe_parse": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_lhe_read_error": (ctypes.c_char_p, []),
    "rwgt_lhe_destroy": (None, [ctypes.c_void_p]),
    "rwgt_lhe_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "rwgt_lhe_num_events": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_lhe_event_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "rwgt_lhe_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_double)]),
    "rwgt_lhe_select": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_lhe_momenta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    "rwgt_lhe_add_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_char_p,
                                             ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_double)]),
    "rwgt_lhe_write": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "rwgt_process_layout": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_char_p)]),
    "rwgt_reweight_card": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.c_char_p, ctypes.c_int32, ctypes.c_char_p]),
})

class TrainCfg(ctypes.Structure):
    """rwgt_train_cfg of include/rwgt.h."""
    _fields_ = [("batch", ctypes.c_int64), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("seed", ctypes.c_uint64)]


SIGNATURES.update({
    "rwgt_mlp_get_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_mlp_fit_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rwgt_mlp_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(TrainCfg),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "rwgt_mlp_get_progress": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3),
    "rwgt_train_order": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_mlp_calibrate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_double)]),
    "rwgt_mlp_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "rwgt_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rwgt_mlp_checkpoint_info": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_mlp_checkpoint_error": (ctypes.c_char_p, []),
})

SIGNATURES.update({
    "rwgt_set_mixed_guard": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "rwgt_mixed_guard_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rwgt_cancellation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p]),
})

SIGNATURES["rwgt_xsec"] = (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int32)])
SIGNATURES["rwgt_xsec_noalloc"] = SIGNATURES["rwgt_xsec"]

_lib = None


class RwgtError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


def load():
    """Load librwgt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_05100_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_f64(t, name):
    """A contiguous float64 torch tensor in device or host memory (rwgt_eval
    and rwgt_me2 copy host arrays through the library's staging buffer)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")


def _check_device(t, name, shape_prefix=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")


def _host_params(param_sets):
    a = np.ascontiguousarray(np.asarray(param_sets, dtype=np.float64))
    if a.ndim == 1:
        a = a[None, :]
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _raise(code, ctx=None):
    lib = load()
    msg = lib.rwgt_last_error(ctx) if ctx is not None else lib.rwgt_create_error()
    raise RwgtError(code, (msg or b"").decode())


def rwgt_create(process: str, param_card: str, precision: int = RWGT_FP64):
    lib = load()
    out = ctypes.c_void_p()
    rc = lib.rwgt_create(process.encode(), param_card.encode(), int(precision), ctypes.byref(out))
    if rc != 0:
        _raise(rc)
    return out


def rwgt_destroy(ctx):
    if ctx:
        load().rwgt_destroy(ctx)


def rwgt_param_layout(ctx):
    lib = load()
    n = ctypes.c_int32()
    rc = lib.rwgt_param_layout(ctx, ctypes.byref(n), None)
    if rc != 0:
        _raise(rc, ctx)
    names = (ctypes.c_char_p * n.value)()
    lib.rwgt_param_layout(ctx, ctypes.byref(n), names)
    return [s.decode() for s in names]


def rwgt_original_params(ctx):
    n = len(rwgt_param_layout(ctx))
    out = (ctypes.c_double * n)()
    rc = load().rwgt_original_params(ctx, out)
    if rc != 0:
        _raise(rc, ctx)
    return np.array(out[:], dtype=np.float64)


def rwgt_set_stream(ctx, stream=None):
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None (current torch stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    rc = load().rwgt_set_stream(ctx, ctypes.c_void_p(handle))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_eval(ctx, momenta, weights_in, param_sets, weights_out):
    """weights_out[k, i] = weights_in[i] / |M|^2_orig[i] * |M|^2_k[i] (enqueued on the set stream).
    Tensors on the GPU or in host memory (pinned: still asynchronous;
    pageable: the call waits)."""
    _check_f64(momenta, "momenta")
    _check_f64(weights_in, "weights_in")
    _check_f64(weights_out, "weights_out")
    nevt = momenta.shape[0] if momenta.dim() > 0 else 0
    params, pptr = _host_params(param_sets)
    if weights_out.numel() != params.shape[0] * nevt or weights_in.numel() != nevt:
        raise ValueError("weights_in must be [nevt] and weights_out [nsets, nevt]")
    rc = load().rwgt_eval(ctx, _ptr(momenta), nevt, _ptr(weights_in), pptr, params.shape[0], _ptr(weights_out))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_eval_alphas(ctx, momenta, weights_in, alphas_orig, scales, param_sets, weights_out):
    """As rwgt_eval with the strong coupling per event (alphas_orig may be None)."""
    _check_device(momenta, "momenta")
    _check_device(weights_in, "weights_in")
    _check_device(scales, "scales")
    _check_device(weights_out, "weights_out")
    if alphas_orig is not None:
        _check_device(alphas_orig, "alphas_orig")
    nevt = momenta.shape[0] if momenta.dim() > 0 else 0
    params, pptr = _host_params(param_sets)
    if weights_out.numel() != params.shape[0] * nevt or weights_in.numel() != nevt or scales.numel() != nevt:
        raise ValueError("weights_in and scales must be [nevt] and weights_out [nsets, nevt]")
    rc = load().rwgt_eval_alphas(ctx, _ptr(momenta), nevt, _ptr(weights_in),
                                 None if alphas_orig is None else _ptr(alphas_orig), _ptr(scales), pptr,
                                 params.shape[0], _ptr(weights_out))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_eval_factored(ctx, momenta, weights_in, param_sets, weights_out):
    """As rwgt_eval, through the coupling-factored path."""
    _check_device(momenta, "momenta")
    _check_device(weights_in, "weights_in")
    _check_device(weights_out, "weights_out")
    nevt = momenta.shape[0] if momenta.dim() > 0 else 0
    params, pptr = _host_params(param_sets)
    if weights_out.numel() != params.shape[0] * nevt or weights_in.numel() != nevt:
        raise ValueError("weights_in must be [nevt] and weights_out [nsets, nevt]")
    rc = load().rwgt_eval_factored(ctx, _ptr(momenta), nevt, _ptr(weights_in), pptr, params.shape[0],
                                   _ptr(weights_out))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_me2(ctx, momenta, param_sets, me2_out):
    """me2_out[k, i] = |M|^2_k[i]; tensors on the GPU or in host memory, as rwgt_eval."""
    _check_f64(momenta, "momenta")
    _check_f64(me2_out, "me2_out")
    nevt = momenta.shape[0]
    params, pptr = _host_params(param_sets)
    if me2_out.numel() != params.shape[0] * nevt:
        raise ValueError("me2_out must be [nsets, nevt]")
    rc = load().rwgt_me2(ctx, _ptr(momenta), nevt, pptr, params.shape[0], _ptr(me2_out))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_nonfinite(ctx):
    """Non-finite outputs of the last evaluation on ctx (waits for it)."""
    out = ctypes.c_int64()
    rc = load().rwgt_nonfinite(ctx, ctypes.byref(out))
    if rc != 0:
        _raise(rc, ctx)
    return out.value


def rwgt_process_info(ctx):
    vals = [ctypes.c_int32() for _ in range(4)]
    rc = load().rwgt_process_info(ctx, *[ctypes.byref(v) for v in vals])
    if rc != 0:
        _raise(rc, ctx)
    return dict(zip(("npart", "nhel_kept", "ncol", "ndiag"), (v.value for v in vals)))


def rwgt_flops(ctx):
    out = ctypes.c_double()
    rc = load().rwgt_flops(ctx, ctypes.byref(out))
    if rc != 0:
        _raise(rc, ctx)
    return out.value


def rwgt_bounds_check():
    """(enabled, misses): whether this is the bounds-checked build, and the
    out-of-range device indices counted since the previous call."""
    en, n = ctypes.c_int32(), ctypes.c_uint64()
    rc = load().rwgt_bounds_check(ctypes.byref(en), ctypes.byref(n))
    if rc != 0:
        _raise(rc, None)
    return bool(en.value), int(n.value)


def rwgt_flops_executed(ctx):
    out = ctypes.c_double()
    rc = load().rwgt_flops_executed(ctx, ctypes.byref(out))
    if rc != 0:
        _raise(rc, ctx)
    return out.value


def rwgt_set_profiling(ctx, enable=True):
    rc = load().rwgt_set_profiling(ctx, int(bool(enable)))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_kernel_times(ctx):
    """(ingest_ms, me_ms) of the last call made with profiling on."""
    a, b = ctypes.c_float(), ctypes.c_float()
    rc = load().rwgt_kernel_times(ctx, ctypes.byref(a), ctypes.byref(b))
    if rc != 0:
        _raise(rc, ctx)
    return a.value, b.value


def _braise(code, batch):
    raise RwgtError(code, (load().rwgt_batch_last_error(batch) or b"").decode())


def rwgt_batch_create(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    out = ctypes.c_void_p()
    rc = load().rwgt_batch_create(arr, len(ctxs), ctypes.byref(out))
    if rc != 0:
        raise RwgtError(rc, "rwgt_batch_create failed")
    return out


def rwgt_batch_destroy(batch):
    if batch:
        load().rwgt_batch_destroy(batch)


def rwgt_batch_set_stream(batch, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    rc = load().rwgt_batch_set_stream(batch, ctypes.c_void_p(handle))
    if rc != 0:
        _braise(rc, batch)


def make_segments(items):
    """items: iterable of (ctx_index, momenta, weights_in, params row, weights_out);
    returns (ctypes array, keep-alive list)."""
    items = list(items)
    arr = (Segment * len(items))()
    keep = []
    for s, (ci, mom, w_in, params, w_out) in zip(arr, items):
        for t, name in ((mom, "momenta"), (w_in, "weights_in"), (w_out, "weights_out")):
            _check_device(t, name)
        prow, pptr = _host_params(params)
        keep.append(prow)
        s.ctx, s.nevt = int(ci), int(mom.shape[0])
        s.momenta, s.weights_in, s.weights_out = mom.data_ptr(), w_in.data_ptr(), w_out.data_ptr()
        s.params = pptr
    return arr, keep


def _segment_array(segments):
    if isinstance(segments, ctypes.Array):
        return segments
    segments = list(segments)
    return (Segment * len(segments))(*segments)


def rwgt_batch_eval(batch, segments):
    segments = _segment_array(segments)
    rc = load().rwgt_batch_eval(batch, segments, len(segments))
    if rc != 0:
        _braise(rc, batch)


def rwgt_batch_time(batch):
    ms = ctypes.c_float()
    rc = load().rwgt_batch_time(batch, ctypes.byref(ms))
    if rc != 0:
        _braise(rc, batch)
    return ms.value


def rwgt_batch_set_schedule(batch, tile_events, block, blocks_per_cu, hel_split=0):
    rc = load().rwgt_batch_set_schedule(batch, tile_events, block, blocks_per_cu, int(hel_split))
    if rc != 0:
        _braise(rc, batch)


def rwgt_batch_get_schedule(batch):
    v = [ctypes.c_int32() for _ in range(4)]
    rc = load().rwgt_batch_get_schedule(batch, *[ctypes.byref(x) for x in v])
    if rc != 0:
        _braise(rc, batch)
    return dict(zip(("tile_events", "block", "grid", "hel_split"), (x.value for x in v)))


def rwgt_batch_tune(batch, segments, reps=2):
    segments = _segment_array(segments)
    rc = load().rwgt_batch_tune(batch, segments, len(segments), reps)
    if rc != 0:
        _braise(rc, batch)
    return rwgt_batch_get_schedule(batch)


# ------------------------------------------------------------------ surrogate
RWGT_MLP_BF16, RWGT_MLP_FP32 = 0, 1
RWGT_FEAT_RAW, RWGT_FEAT_PHYS = 0, 1


def n_features(kind, npart):
    """Width of a feature map (rwgt_mlp_set_features)."""
    return npart * 4 + 3 if kind == RWGT_FEAT_RAW else 1 + npart * (npart - 1) // 2 + 3 + 4


def _mraise(code, mlp):
    raise RwgtError(code, (load().rwgt_mlp_last_error(mlp) or b"").decode())


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def rwgt_mlp_create(n_in, width, depth, n_out=2, precision=RWGT_MLP_BF16, seed=0):
    out = ctypes.c_void_p()
    rc = load().rwgt_mlp_create(n_in, width, depth, n_out, precision, seed, ctypes.byref(out))
    if rc != 0:
        raise RwgtError(rc, "rwgt_mlp_create failed")
    return out


def rwgt_mlp_destroy(mlp):
    if mlp:
        load().rwgt_mlp_destroy(mlp)


def rwgt_mlp_set_stream(mlp, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    rc = load().rwgt_mlp_set_stream(mlp, ctypes.c_void_p(handle))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_num_params(mlp):
    n = ctypes.c_int64()
    rc = load().rwgt_mlp_num_params(mlp, ctypes.byref(n))
    if rc != 0:
        _mraise(rc, mlp)
    return n.value


def rwgt_mlp_get_params(mlp):
    out = np.zeros(rwgt_mlp_num_params(mlp), dtype=np.float32)
    rc = load().rwgt_mlp_get_params(mlp, _fptr(out))
    if rc != 0:
        _mraise(rc, mlp)
    return out


def rwgt_mlp_set_params(mlp, flat):
    a = np.ascontiguousarray(flat, dtype=np.float32)
    rc = load().rwgt_mlp_set_params(mlp, _fptr(a))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_get_grads(mlp):
    out = np.zeros(rwgt_mlp_num_params(mlp), dtype=np.float32)
    rc = load().rwgt_mlp_get_grads(mlp, _fptr(out))
    if rc != 0:
        _mraise(rc, mlp)
    return out


def rwgt_mlp_set_normalisation(mlp, mean, std):
    m = np.ascontiguousarray(mean, dtype=np.float32)
    s = np.ascontiguousarray(std, dtype=np.float32)
    rc = load().rwgt_mlp_set_normalisation(mlp, _fptr(m), _fptr(s))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_set_features(mlp, kind, npart, res=(2, 3), orig=(0.0, 0.0)):
    rc = load().rwgt_mlp_set_features(mlp, int(kind), int(npart), int(res[0]), int(res[1]), float(orig[0]),
                                      float(orig[1]))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_set_target_scale(mlp, mean, std):
    rc = load().rwgt_mlp_set_target_scale(mlp, float(mean), float(std))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_fit_normalisation(mlp, momenta, event_index, card_index, card_params, n):
    rc = load().rwgt_mlp_fit_normalisation(mlp, _dp(momenta), momenta.shape[1], _dp(event_index), _dp(card_index),
                                           _dp(card_params), int(n))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_get_normalisation(mlp, n_in):
    """(mean [n_in], std [n_in], (y_mean, y_std))."""
    mean = np.zeros(n_in, dtype=np.float32)
    std = np.zeros(n_in, dtype=np.float32)
    ys = np.zeros(2, dtype=np.float32)
    rc = load().rwgt_mlp_get_normalisation(mlp, _fptr(mean), _fptr(std), _fptr(ys))
    if rc != 0:
        _mraise(rc, mlp)
    return mean, std, (float(ys[0]), float(ys[1]))


def rwgt_mlp_fit_target_scale(mlp, y, n=None):
    rc = load().rwgt_mlp_fit_target_scale(mlp, _dp(y), int(y.numel() if n is None else n))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_set_training(mlp, lam=0.1, beta1=0.9, beta2=0.999, eps=1e-8):
    rc = load().rwgt_mlp_set_training(mlp, lam, beta1, beta2, eps)
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_set_calibration(mlp, k):
    rc = load().rwgt_mlp_set_calibration(mlp, float(k))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_input_bytes(mlp, n):
    b = ctypes.c_int64()
    rc = load().rwgt_mlp_input_bytes(mlp, int(n), ctypes.byref(b))
    if rc != 0:
        _mraise(rc, mlp)
    return b.value


def _dp(t):
    return ctypes.c_void_p(0) if t is None else ctypes.c_void_p(t.data_ptr())


def rwgt_mlp_features(mlp, momenta, event_index, card_index, card_params, n, x_out):
    """momenta: [nev, npart, 4] f64; event_index/card_index: int32 [n] (event_index may be None);
    card_params: f32 [ncards, nparam]; x_out: device buffer (uint8 tensor of rwgt_mlp_input_bytes)."""
    rc = load().rwgt_mlp_features(mlp, _dp(momenta), momenta.shape[1], _dp(event_index), _dp(card_index),
                                  _dp(card_params), card_params.shape[1], int(n), _dp(x_out))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_forward(mlp, x, n, heads_out=None):
    rc = load().rwgt_mlp_forward(mlp, _dp(x), int(n), _dp(heads_out))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_predict(mlp, momenta, event_index, card_index, card_params, n, heads_out):
    """Fused forward pass: heads_out [n, 2] f32 (mu, s) for rows (event_index[r] or r, card_index[r])."""
    rc = load().rwgt_mlp_predict(mlp, _dp(momenta), momenta.shape[1], _dp(event_index), _dp(card_index),
                                 _dp(card_params), int(n), _dp(heads_out))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_train_step(mlp, x, y, n, lr, loss_out=None):
    rc = load().rwgt_mlp_train_step(mlp, _dp(x), _dp(y), int(n), float(lr), _dp(loss_out))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_targets(mlp, w_new, w_old, y):
    rc = load().rwgt_mlp_targets(mlp, _dp(w_new), _dp(w_old), int(w_new.numel()), _dp(y))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_eval_cards(ctx, momenta, weights_in, param_table, card_index, weights_out):
    """Exact w' with a card per event: weights_out[i] under param_table[card_index[i]]."""
    _check_device(momenta, "momenta")
    _check_device(weights_in, "weights_in")
    _check_device(weights_out, "weights_out")
    table, tptr = _host_params(param_table)
    rc = load().rwgt_eval_cards(ctx, _dp(momenta), momenta.shape[0], _dp(weights_in), tptr, table.shape[0],
                                _dp(card_index), _dp(weights_out))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_sur_eval(ctx, mlp, momenta, weights_in, param_table, card_index, err_threshold, weights_out):
    """Returns the number of events that took the exact path."""
    _check_device(momenta, "momenta")
    _check_device(weights_in, "weights_in")
    _check_device(weights_out, "weights_out")
    table, tptr = _host_params(param_table)
    nfb = ctypes.c_int64()
    rc = load().rwgt_sur_eval(ctx, mlp, _dp(momenta), momenta.shape[0], _dp(weights_in), tptr, table.shape[0],
                              _dp(card_index), float(err_threshold), _dp(weights_out), ctypes.byref(nfb))
    if rc != 0:
        _raise(rc, ctx)
    return nfb.value


def rwgt_xsec(ctx, weights_in, weights_out, sigma, dsigma, norm, entry="rwgt_xsec"):
    """(sigma'[k], dsigma'[k], fallback[k]) for weights_out [nsets, nevt]
    (entry "rwgt_xsec_noalloc": the same through the no-allocation entry point)."""
    _check_device(weights_in, "weights_in")
    _check_device(weights_out, "weights_out")
    nsets, nevt = weights_out.shape
    xs = np.zeros(nsets)
    xe = np.zeros(nsets)
    fb = np.zeros(nsets, dtype=np.int32)
    rc = getattr(load(), entry)(ctx, _dp(weights_in), _dp(weights_out), nevt, nsets, sigma, dsigma, norm,
                          xs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          xe.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        _raise(rc, ctx)
    return xs, xe, fb.astype(bool)


# ----------------------------------------------------------------- event files
def _lraise(code, lhe):
    raise RwgtError(code, (load().rwgt_lhe_last_error(lhe) or b"").decode())


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def rwgt_lhe_read(path):
    out = ctypes.c_void_p()
    rc = load().rwgt_lhe_read(str(path).encode(), ctypes.byref(out))
    if rc != 0:
        raise RwgtError(rc, (load().rwgt_lhe_read_error() or b"").decode())
    return out


def rwgt_lhe_parse(text):
    data = text.encode() if isinstance(text, str) else bytes(text)
    out = ctypes.c_void_p()
    rc = load().rwgt_lhe_parse(data, len(data), ctypes.byref(out))
    if rc != 0:
        raise RwgtError(rc, (load().rwgt_lhe_read_error() or b"").decode())
    return out


def rwgt_lhe_destroy(lhe):
    if lhe:
        load().rwgt_lhe_destroy(lhe)


def rwgt_lhe_num_events(lhe):
    n = ctypes.c_int64()
    rc = load().rwgt_lhe_num_events(lhe, ctypes.byref(n))
    if rc != 0:
        _lraise(rc, lhe)
    return n.value


def rwgt_lhe_event_info(lhe, i):
    """(nup, idprup, (XWGTUP, SCALUP, AQEDUP, AQCDUP))."""
    nup, idp = ctypes.c_int32(), ctypes.c_int32()
    info = np.zeros(4)
    rc = load().rwgt_lhe_event_info(lhe, int(i), ctypes.byref(nup), ctypes.byref(idp), _f64(info))
    if rc != 0:
        _lraise(rc, lhe)
    return nup.value, idp.value, tuple(float(x) for x in info)


def rwgt_lhe_info(lhe, index):
    """[n, 4] host array of (XWGTUP, SCALUP, AQEDUP, AQCDUP)."""
    index = np.ascontiguousarray(index, dtype=np.int64)
    out = np.zeros((max(index.size, 1), 4))
    rc = load().rwgt_lhe_info(lhe, _i64(index), index.size, _f64(out))
    if rc != 0:
        _lraise(rc, lhe)
    return out[:index.size]


def rwgt_lhe_select(lhe, process):
    """Indices (int64 array) of the events of a process."""
    n = ctypes.c_int64()
    rc = load().rwgt_lhe_select(lhe, process.encode(), None, 0, ctypes.byref(n))
    if rc != 0:
        _lraise(rc, lhe)
    idx = np.zeros(max(n.value, 1), dtype=np.int64)
    rc = load().rwgt_lhe_select(lhe, process.encode(), _i64(idx), n.value, ctypes.byref(n))
    if rc != 0:
        _lraise(rc, lhe)
    return idx[:n.value]


def rwgt_lhe_momenta(lhe, process, index):
    """(momenta [n, npart, 4] (E, px, py, pz), XWGTUP [n]) as host arrays."""
    index = np.ascontiguousarray(index, dtype=np.int64)
    npart = len(process.replace(">", " ").split())
    mom = np.zeros((max(index.size, 1), npart, 4))
    w = np.zeros(max(index.size, 1))
    rc = load().rwgt_lhe_momenta(lhe, process.encode(), _i64(index), index.size, _f64(mom), _f64(w))
    if rc != 0:
        _lraise(rc, lhe)
    return mom[:index.size], w[:index.size]


def rwgt_lhe_add_weights(lhe, weight_id, description, index, w):
    index = np.ascontiguousarray(index, dtype=np.int64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if index.size != w.size:
        raise ValueError("index and weights differ in length")
    rc = load().rwgt_lhe_add_weights(lhe, weight_id.encode(), (description or "").encode(), _i64(index), index.size,
                                     _f64(w))
    if rc != 0:
        _lraise(rc, lhe)


def rwgt_lhe_write(lhe, path):
    rc = load().rwgt_lhe_write(lhe, str(path).encode())
    if rc != 0:
        _lraise(rc, lhe)


def rwgt_process_layout(process):
    """Names of the columns of a process's param_sets rows."""
    n = ctypes.c_int32()
    rc = load().rwgt_process_layout(process.encode(), ctypes.byref(n), None)
    if rc != 0:
        raise RwgtError(rc, f"unsupported process '{process}'")
    names = (ctypes.c_char_p * n.value)()
    load().rwgt_process_layout(process.encode(), ctypes.byref(n), names)
    return [x.decode() for x in names]


def rwgt_reweight_card(process, param_card, rwgt_card, cap=4096, name_len=64):
    """(param_sets [nsets, npar], names [nsets], fptype or None) from a reweighting card."""
    npar = len(rwgt_process_layout(process))
    buf = np.zeros((cap, npar))
    n = ctypes.c_int32()
    names = ctypes.create_string_buffer(cap * name_len)
    fp = ctypes.create_string_buffer(2)
    rc = load().rwgt_reweight_card(process.encode(), param_card.encode(), rwgt_card.encode(), cap, _f64(buf),
                                   ctypes.byref(n), names, name_len, fp)
    if rc != 0:
        raise RwgtError(rc, (load().rwgt_create_error() or b"").decode())
    if n.value > cap:
        return rwgt_reweight_card(process, param_card, rwgt_card, cap=n.value, name_len=name_len)
    out_names = [names.raw[i * name_len:(i + 1) * name_len].split(b"\0")[0].decode() for i in range(n.value)]
    return buf[:n.value], out_names, (fp.value.decode() or None)


# ------------------------------------------------------- training on a grid
def rwgt_mlp_get_adam(mlp):
    """(first moments, second moments, Adam steps) packed as rwgt_mlp_get_params."""
    n = rwgt_mlp_num_params(mlp)
    first, second = np.zeros(n, dtype=np.float32), np.zeros(n, dtype=np.float32)
    steps = ctypes.c_int64()
    rc = load().rwgt_mlp_get_adam(mlp, _fptr(first), _fptr(second), ctypes.byref(steps))
    if rc != 0:
        _mraise(rc, mlp)
    return first, second, steps.value


def rwgt_mlp_fit_grid(mlp, momenta, card_params, y):
    """momenta [nevt, npart, 4] f64, card_params [ncards, 3] f32, y [ncards, nevt] f32 (device)."""
    rc = load().rwgt_mlp_fit_grid(mlp, _dp(momenta), momenta.shape[1], momenta.shape[0], _dp(card_params),
                                  card_params.shape[0], _dp(y))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_train(mlp, momenta, card_params, y, batch, epochs, lr, lr_final, seed, epoch_end):
    """Train epochs [done, epoch_end) of the schedule; returns the mean loss per pair of each."""
    cfg = TrainCfg(int(batch), int(epochs), float(lr), float(lr_final), int(seed))
    done, _, _ = rwgt_mlp_get_progress(mlp)
    losses = np.zeros(max(int(epoch_end) - done, 0), dtype=np.float32)
    rc = load().rwgt_mlp_train(mlp, _dp(momenta), momenta.shape[1], momenta.shape[0], _dp(card_params),
                               card_params.shape[0], _dp(y), ctypes.byref(cfg), int(epoch_end), _fptr(losses))
    if rc != 0:
        _mraise(rc, mlp)
    return losses


def rwgt_mlp_get_progress(mlp):
    """(epochs done, schedule steps done, Adam steps taken)."""
    vals = [ctypes.c_int64() for _ in range(3)]
    rc = load().rwgt_mlp_get_progress(mlp, *[ctypes.byref(v) for v in vals])
    if rc != 0:
        _mraise(rc, mlp)
    return tuple(v.value for v in vals)


def rwgt_train_order(seed, epoch, n, pos0=0, count=None):
    count = n - pos0 if count is None else count
    out = np.zeros(count, dtype=np.int64)
    rc = load().rwgt_train_order(int(seed), int(epoch), int(n), int(pos0), int(count),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RwgtError(rc, "rwgt_train_order: bad arguments")
    return out


def rwgt_mlp_calibrate(mlp, momenta, card_params, y, coverage):
    """(k, median |r|, 0.9 quantile of |r|, 0.999 quantile of |r|); sets the network's k."""
    stats = np.zeros(4)
    rc = load().rwgt_mlp_calibrate(mlp, _dp(momenta), momenta.shape[1], momenta.shape[0], _dp(card_params),
                                   card_params.shape[0], _dp(y), float(coverage),
                                   stats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        _mraise(rc, mlp)
    return tuple(float(v) for v in stats)


def _ckraise(code):
    raise RwgtError(code, (load().rwgt_mlp_checkpoint_error() or b"").decode())


def rwgt_mlp_save(mlp, path):
    rc = load().rwgt_mlp_save(mlp, os.fsencode(path))
    if rc != 0:
        _mraise(rc, mlp)


def rwgt_mlp_load(path):
    out = ctypes.c_void_p()
    rc = load().rwgt_mlp_load(os.fsencode(path), ctypes.byref(out))
    if rc != 0:
        _ckraise(rc)
    return out


def rwgt_mlp_checkpoint_info(path):
    """((n_in, width, depth, n_out, precision), epochs done, Adam steps); host only."""
    shape = (ctypes.c_int32 * 5)()
    epoch, steps = ctypes.c_int64(), ctypes.c_int64()
    rc = load().rwgt_mlp_checkpoint_info(os.fsencode(path), shape, ctypes.byref(epoch), ctypes.byref(steps))
    if rc != 0:
        _ckraise(rc)
    return tuple(shape), epoch.value, steps.value


# ------------------------------------------------------ mixed-path guard
def rwgt_set_mixed_guard(ctx, kappa_max):
    rc = load().rwgt_set_mixed_guard(ctx, float(kappa_max))
    if rc != 0:
        _raise(rc, ctx)


def rwgt_mixed_guard_count(ctx):
    n = ctypes.c_int64()
    rc = load().rwgt_mixed_guard_count(ctx, ctypes.byref(n))
    if rc != 0:
        _raise(rc, ctx)
    return n.value


def rwgt_cancellation(ctx, momenta, param_sets, kappa_out, me2_out=None):
    """Mixed |M|^2 (optional, [nsets, nevt]) and kappa [nevt] per event, without re-evaluation."""
    _check_device(momenta, "momenta")
    _check_device(kappa_out, "kappa_out")
    a, ptr = _host_params(param_sets)
    rc = load().rwgt_cancellation(ctx, _ptr(momenta), momenta.shape[0], ptr, a.shape[0], _ptr(me2_out),
                                  _ptr(kappa_out))
    if rc != 0:
        _raise(rc, ctx)
