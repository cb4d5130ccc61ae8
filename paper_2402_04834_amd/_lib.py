"""ctypes binding of libbbp.so (argument marshalling only; every step of the decoder runs in the library).

Names follow the C ABI of include/bbp.h. The library must have been built in-tree
(`python -m paper_2402_04834_amd.build`); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbbp.so")

BBP_OK = 0
BBP_EINVAL = -1
BBP_ENOMEM = -2
BBP_EHIP = -3
BBP_EUNSUPPORTED = -4


class bbp_opts(C.Structure):
    _fields_ = [
        ("block_rows", C.c_int32), ("block_cols", C.c_int32), ("chi", C.c_int32), ("max_iter", C.c_int32),
        ("delta0", C.c_double), ("delta1", C.c_double), ("damping", C.c_double),
        ("rule", C.c_int32), ("fixed_iters", C.c_int32), ("precision", C.c_int32), ("graph", C.c_int32),
        ("gate", C.c_double),
    ]


class bbp_group(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("chi", C.c_int32), ("p", C.c_double), ("p_dev", C.c_void_p),
        ("syndromes_dev", C.c_void_p), ("batch", C.c_int64),
        ("loglik_dev", C.c_void_p), ("delta_dev", C.c_void_p), ("iters_dev", C.c_void_p),
        ("coset_dev", C.c_void_p), ("correction_dev", C.c_void_p), ("init_messages_dev", C.c_void_p),
        ("messages_dev", C.c_void_p), ("noise", C.c_double * 4),
    ]


class bbp_tuning(C.Structure):
    _fields_ = [("order", C.c_int32), ("streams", C.c_int32), ("ms", C.c_double)]


class bbp_plan_info(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("n", C.c_int32), ("m", C.c_int32),
        ("block_grid_rows", C.c_int32), ("block_grid_cols", C.c_int32),
        ("num_messages", C.c_int32), ("updates_per_iter", C.c_int32), ("exact_sweeps", C.c_int32),
        ("max_cut_rank", C.c_int32), ("gpu_supported", C.c_int32),
        ("flops_per_iter", C.c_double), ("flops_bethe", C.c_double),
        ("truncating_sweeps", C.c_int32), ("message_stride", C.c_int32),
    ]


class bbp_timing(C.Structure):
    _fields_ = [
        ("update_ms", C.c_double), ("update_launches", C.c_int32), ("bethe_ms", C.c_double),
        ("other_ms", C.c_double), ("update_flops", C.c_double),
        ("top_class", C.c_int32), ("top_launches", C.c_int32), ("top_ms", C.c_double), ("top_flops", C.c_double),
    ]


TRUNC_CLASS = 1 << 12   # class code of the truncating block sweeps (trunc_sweep.hip); | 1: their narrow form


def is_trunc_class(cls: int) -> bool:
    return (cls & ~1) == TRUNC_CLASS


def sweep_kernel_name(cls: int, precision: int = 0) -> str:
    """Kernel instantiation of a sweep class code (see bbp_timing.top_class): sweep_kernel<...> for FP32,
    sweep_kernel_bf16<...> for the BF16 matrix-core variant of precision mode 1, trunc_sweep_kernel for the
    truncating sweeps (FP64 at either precision; <true> the narrow form, chi <= 8 and at most 7 positions)."""
    if is_trunc_class(cls):
        return f"trunc_sweep_kernel<{'true' if cls & 1 else 'false'}>"
    q00, single, bot, top, kt = cls & 1, (cls >> 1) & 1, (cls >> 2) & 1, (cls >> 3) & 1, (cls >> 4) + 1
    b = lambda v: "true" if v else "false"
    return f"sweep_kernel{'_bf16' if precision else ''}<{kt}, {b(top)}, {b(bot)}, {b(single)}, {b(q00)}>"


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "bbp_default_opts": (None, [C.POINTER(bbp_opts)]),
    "bbp_last_error": (C.c_char_p, []),
    "bbp_build_network": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "bbp_net_dims": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "bbp_net_labels": (C.c_int, [C.c_void_p, C.c_void_p]),
    "bbp_free_network": (None, [C.c_void_p]),
    "bbp_plan_query": (C.c_int, [C.c_int32, C.POINTER(bbp_opts), C.POINTER(bbp_plan_info)]),
    "bbp_workspace_size": (C.c_int, [C.c_int32, C.c_int64, C.POINTER(bbp_opts), C.POINTER(C.c_size_t)]),
    "bbp_decode_device": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.POINTER(bbp_opts),
                                    C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(bbp_timing)]),
    "bbp_decode_device_noalloc": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.POINTER(bbp_opts),
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "bbp_noalloc_max_batch": (C.c_int, [C.c_int32, C.POINTER(bbp_opts), C.POINTER(C.c_int64)]),
    "bbp_workspace_size_groups": (C.c_int, [C.POINTER(bbp_group), C.c_int32, C.POINTER(bbp_opts),
                                            C.POINTER(C.c_size_t)]),
    "bbp_decode_groups": (C.c_int, [C.POINTER(bbp_group), C.c_int32, C.POINTER(bbp_opts), C.c_void_p, C.c_size_t,
                                    C.c_void_p, C.POINTER(bbp_timing)]),
    "bbp_autotune": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_int64, C.POINTER(bbp_opts), C.c_void_p,
                               C.c_size_t, C.c_void_p, C.POINTER(bbp_tuning)]),
    "bbp_set_tuning": (C.c_int, [C.c_int32, C.POINTER(bbp_opts), C.POINTER(bbp_tuning)]),
    "bbp_blockbp_decode": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(bbp_opts), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "bbp_reference_update_host": (C.c_int, [C.c_int32, C.c_double, C.POINTER(bbp_opts), C.c_void_p, C.c_int32,
                                            C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "bbp_bmps_workspace_size": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "bbp_bmps_decode_device": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.POINTER(C.c_float)]),
    "bbp_warm_last_error": (C.c_char_p, []),
    "bbp_warm_param_count": (C.c_int, [C.POINTER(C.c_int64)]),
    "bbp_warm_workspace_size": (C.c_int, [C.c_int32, C.c_int64, C.POINTER(bbp_opts), C.c_int32,
                                          C.POINTER(C.c_size_t)]),
    "bbp_warm_predict": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(bbp_opts),
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "bbp_warm_loss_grad": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(bbp_opts),
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_size_t, C.c_void_p]),
    "bbp_warm_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p]),
    "bbp_warm_decode_workspace_size": (C.c_int, [C.c_int32, C.c_int64, C.POINTER(bbp_opts), C.POINTER(C.c_size_t)]),
    "bbp_warm_decode": (C.c_int, [C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(bbp_opts),
                                  C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library (loads it on first use; raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_04834_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


class BbpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbbp error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != BBP_OK:
        raise BbpError(rc, lib().bbp_last_error().decode())
    return rc


def check_warm(rc):
    """check() for the warm-start entry points, which keep their own error message."""
    if rc != BBP_OK:
        raise BbpError(rc, lib().bbp_warm_last_error().decode())
    return rc


def default_opts(**kw) -> bbp_opts:
    o = bbp_opts()
    lib().bbp_default_opts(C.byref(o))
    for k, v in kw.items():
        if k in ("block", "blocks"):
            o.block_rows, o.block_cols = (v, v) if isinstance(v, int) else v
        else:
            setattr(o, k, v)
    return o
