"""ctypes declarations of the salprior C-ABI (include/salprior.h).

Loading fails loudly when the built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsalprior.so")

SP_OK, SP_EINVAL, SP_ESHAPE, SP_ENOMEM, SP_EHIP, SP_ESTATE = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {SP_EINVAL: "SP_EINVAL", SP_ESHAPE: "SP_ESHAPE", SP_ENOMEM: "SP_ENOMEM",
               SP_EHIP: "SP_EHIP", SP_ESTATE: "SP_ESTATE"}
MAX_LEVELS = 12
NKINDS = 29

c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t


class sp_params(ctypes.Structure):
    _fields_ = [
        ("depth", c_int32),
        ("n_centers", c_int32),
        ("centers", c_int32 * 4),
        ("n_deltas", c_int32),
        ("deltas", c_int32 * 4),
        ("weights", c_float * 8),
        ("q", c_double),
        ("r", c_double),
        ("eps", c_float),
        ("border", c_int32),
        ("lambda_", c_float),
        ("potts", c_float),
        ("lm_block", c_int32),
        ("flat_tol", c_float),
        ("gabor_lambda", c_float),
        ("gabor_sigma", c_float),
        ("gabor_radius", c_int32),
        ("record_tape", c_int32),
        ("f_mode", c_int32),
        ("dt_sigma", c_float),
        ("ssm_q", c_double),
        ("ssm_r", c_double),
        ("gmm_components", c_int32),
        ("gmm_iters", c_int32),
        ("gmm_reg", c_float),
    ]


class sp_geometry(ctypes.Structure):
    _fields_ = [
        ("H", c_int32), ("W", c_int32), ("depth", c_int32), ("top", c_int32),
        ("c_min", c_int32), ("c_max", c_int32), ("n_pairs", c_int32),
        ("pair_c", c_int32 * 16), ("pair_s", c_int32 * 16),
        ("level_h", c_int32 * (MAX_LEVELS + 1)), ("level_w", c_int32 * (MAX_LEVELS + 1)),
        ("Hc", c_int32), ("Wc", c_int32),
    ]


# (name, restype, argtypes) of every exported symbol, in header order.
SIGNATURES = [
    ("sp_default_params", None, [ctypes.POINTER(sp_params)]),
    ("sp_create", c_int32, [ctypes.POINTER(sp_params), c_int32, c_int32, c_void_p, ctypes.POINTER(c_void_p)]),
    ("sp_destroy", c_int32, [c_void_p]),
    ("sp_set_stream", c_int32, [c_void_p, c_void_p]),
    ("sp_get_geometry", c_int32, [c_void_p, ctypes.POINTER(sp_geometry)]),
    ("sp_set_weights", c_int32, [c_void_p, ctypes.POINTER(c_float), c_double, c_double]),
    ("sp_reset", c_int32, [c_void_p]),
    ("sp_step_index", ctypes.c_int64, [c_void_p]),
    ("sp_tape_generation", ctypes.c_int64, [c_void_p]),
    ("saliency_forward", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("prior_update", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("sp_manual_prior", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("sp_stochastic_saliency", c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_double)]),
    ("mrf_weights", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("sp_colour_likelihood", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("sp_cut_create", c_int32, [c_int32, c_int32, c_void_p, ctypes.POINTER(c_void_p)]),
    ("sp_cut_destroy", c_int32, [c_void_p]),
    ("sp_mincut", c_int32, [c_void_p, c_void_p, c_void_p, c_float, c_void_p, c_void_p]),
    ("sp_step", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                          c_void_p, c_void_p]),
    ("saliency_backward", c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    ("saliency_backward_frames", c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    ("sp_mse_mask_loss", c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    ("sp_state_size", c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    ("sp_get_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("sp_set_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("sp_batch_create", c_int32, [ctypes.POINTER(sp_params), c_int32, ctypes.POINTER(c_int32),
                                  ctypes.POINTER(c_int32), c_int32, c_void_p, ctypes.POINTER(c_void_p)]),
    ("sp_batch_step", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("sp_batch_steps", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    ("sp_batch_prior", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    ("sp_batch_outputs", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                   ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    ("sp_batch_consp", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    ("sp_batch_reset", c_int32, [c_void_p]),
    ("sp_batch_destroy", c_int32, [c_void_p]),
    ("sp_batch_set_weights", c_int32, [c_void_p, ctypes.POINTER(c_float), c_double, c_double]),
    ("sp_batch_step_index", ctypes.c_int64, [c_void_p]),
    ("sp_batch_tape_generation", ctypes.c_int64, [c_void_p]),
    ("sp_batch_tape_prior", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p)]),
    ("sp_batch_mse_mask_loss", c_int32, [c_void_p, ctypes.POINTER(c_void_p), c_int32, c_void_p,
                                         ctypes.POINTER(c_void_p)]),
    ("sp_batch_backward", c_int32, [c_void_p, ctypes.POINTER(c_void_p), c_int32, c_void_p, c_void_p, c_void_p]),
    ("sp_profile_enable", c_int32, [c_void_p, c_int32]),
    ("sp_profile_read", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_float), ctypes.POINTER(c_int32)]),
    ("sp_batch_autotune", c_int32, [c_void_p, c_void_p, c_int32, ctypes.c_char_p, c_size_t]),
    ("sp_autotune", c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_char_p, c_size_t]),
    ("sp_batch_profile_enable", c_int32, [c_void_p, c_int32]),
    ("sp_batch_profile_read", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_float), ctypes.POINTER(c_int32)]),
    ("sp_set_tune", c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    ("sp_batch_set_tune", c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    ("sp_tune_cache_clear", c_int32, []),
    ("sp_calibration_copy", c_int32, [c_void_p, c_void_p, c_size_t, c_int32, c_void_p]),
    ("sp_kernel_name", ctypes.c_char_p, [c_int32]),
    ("sp_saliency_noalloc", c_int32, [ctypes.POINTER(sp_params), c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p]),
    ("sp_last_error", ctypes.c_char_p, []),
]

_LIB = None


class SalpriorError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsalprior.so (after torch, so both share one HIP runtime)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"salprior HIP library not built: {path} is missing "
                           "(run `python -m paper_1008_0502_amd.build`)")
    try:
        import torch  # noqa: F401  -- load torch's HIP runtime first
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(rc: int, where: str) -> None:
    if rc != SP_OK:
        msg = _LIB.sp_last_error().decode(errors="replace") if _LIB is not None else ""
        raise SalpriorError(rc, where, msg)


_HIP = None


def hip_copy_d2d(dst: int, src: int, nbytes: int, stream: int) -> None:
    """Device-to-device copy enqueued on `stream` through the HIP runtime torch already
    loaded (moves a library-owned buffer into a caller's tensor; no arithmetic)."""
    global _HIP
    if _HIP is None:
        hip = ctypes.CDLL("libamdhip64.so.7")
        hip.hipMemcpyAsync.restype = ctypes.c_int
        hip.hipMemcpyAsync.argtypes = [c_void_p, c_void_p, c_size_t, ctypes.c_int, c_void_p]
        _HIP = hip
    rc = _HIP.hipMemcpyAsync(dst, src, nbytes, 3, stream)
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")

