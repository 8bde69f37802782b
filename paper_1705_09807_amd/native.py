"""ctypes declarations of the C ABI in include/lbmhd.h and
include/lbmhd_learned.h (liblbmhd.so).

Loading fails loudly when the library has not been built: there is no
fallback implementation.  torch is imported first so that the library binds
to the HIP runtime torch already loaded (both carry the soname
libamdhip64.so.7), which makes torch's streams and device pointers valid in
the library.
"""

from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbmhd.so")
HEADERS = [os.path.join(os.path.dirname(PKG), "include", h) for h in ("lbmhd.h", "lbmhd_learned.h")]

LBM_OK = 0
LBM_EINVAL = -1
LBM_ESTATE = -2
LBM_EHIP = -3
LBM_ENONFINITE = -4

LBM_FP64 = 0
LBM_FP32 = 1
LBM_FP16 = 2
LBM_BF16 = 3
LBM_STENCIL_ISO9 = 0
LBM_STENCIL_CENTRAL5 = 1
LBM_STENCIL_LOCAL_ISO9 = 2
LBM_STENCIL_LOCAL_CENTRAL5 = 3
LBM_SCHED_FUSED = 0
LBM_SCHED_AA = 1
LBM_SCHED_AA_LAGGED = 2
LBM_CLOSURE_ANALYTIC = 0
LBM_CLOSURE_LEARNED = 1
LBM_CLOSURE_FULL = 2
LBM_MAG_D2Q5 = 0
LBM_MAG_D2Q9 = 1

LBM_MLP_FEATURES = 64
LBM_MLP_OUTPUTS = 4
LBM_MLP_OFF_W1 = 0
LBM_MLP_OFF_B1 = 4096
LBM_MLP_OFF_W2 = 4160
LBM_MLP_OFF_B2 = 8256
LBM_MLP_OFF_W3 = 8320
LBM_MLP_OFF_B3 = 8576
LBM_MLP_PARAMS = 8580
LBM_MLP_PACKED_BYTES = 31744
LBM_MLP_TRAIN_NOALLOC_BATCH = 16384
LBM_MLP_TRAIN_NOALLOC_BYTES = 9437184


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nu", ctypes.c_double), ("eta", ctypes.c_double),
        ("s5", ctypes.c_double), ("s6", ctypes.c_double),
        ("s7", ctypes.c_double), ("s8", ctypes.c_double),
        ("delta", ctypes.c_double), ("closure_scale", ctypes.c_double),
        ("grad_stencil", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("schedule", ctypes.c_int32), ("closure", ctypes.c_int32),
        ("mag_lattice", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("rho0", ctypes.c_double),
        ("bref_x", ctypes.c_double), ("bref_y", ctypes.c_double),
    ]


class LbmKhParams(ctypes.Structure):
    _fields_ = [
        ("U0", ctypes.c_double), ("delta_over_L", ctypes.c_double),
        ("B0", ctypes.c_double), ("rho0", ctypes.c_double),
        ("pert_amp_over_U0", ctypes.c_double), ("noise_amp", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class LbmSech2Params(ctypes.Structure):
    _fields_ = [
        ("U0", ctypes.c_double), ("B0", ctypes.c_double), ("pert", ctypes.c_double),
        ("rho0", ctypes.c_double), ("k", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class LbmDiag(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int64),
        ("mass", ctypes.c_double), ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("bsum_x", ctypes.c_double), ("bsum_y", ctypes.c_double),
        ("e_kin", ctypes.c_double), ("e_mag", ctypes.c_double),
        ("enstrophy", ctypes.c_double), ("j2", ctypes.c_double),
        ("divb_max", ctypes.c_double), ("divb_rms", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]


class LbmMlpNorm(ctypes.Structure):
    _fields_ = [
        ("shift", ctypes.c_float * 8), ("scale", ctypes.c_float * 8),
        ("out_scale", ctypes.c_float * 4), ("pad", ctypes.c_float * 12),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_SIGNATURES = {
    "lbm_state_bytes": (ctypes.c_size_t, [ctypes.POINTER(LbmParams)]),
    "lbm_work_bytes": (ctypes.c_size_t, [ctypes.POINTER(LbmParams)]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(LbmParams), _P, _P, _P]),
    "lbm_init_kh_jet": (ctypes.c_int, [_P, ctypes.POINTER(LbmKhParams)]),
    "lbm_init_sech2_jet": (ctypes.c_int, [_P, ctypes.POINTER(LbmSech2Params)]),
    "lbm_init_from_moments": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int64]),
    "lbm_get_time": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_moments": (ctypes.c_int, [_P, _P]),
    "lbm_get_state": (ctypes.c_int, [_P, _P]),
    "lbm_set_state": (ctypes.c_int, [_P, _P, ctypes.c_int64]),
    "lbm_diagnostics": (ctypes.c_int, [_P, ctypes.POINTER(LbmDiag)]),
    "lbm_destroy": (ctypes.c_int, [_P]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_last_error": (ctypes.c_char_p, []),
    # lbmhd_learned.h
    "lbm_mlp_pack": (ctypes.c_int, [_P, _P, _P, _P]),
    "lbm_mlp_forward": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P]),
    "lbm_mlp_stats_work_bytes": (_SZ, [_I64]),
    "lbm_mlp_feature_stats": (ctypes.c_int, [_P, _P, _I64, _P, _P, _SZ, _P]),
    "lbm_mlp_train_work_bytes": (_SZ, [_I32]),
    "lbm_mlp_gradient": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _P, _SZ, _P, _P, _P]),
    "lbm_mlp_adam": (ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.c_double, _P]),
    "lbm_mlp_train_step": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_double, _P, _P, _P, _P, _I32, _P, _SZ, _P, _P]),
    "lbm_mlp_train_step_noalloc": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_double, _P, _P, _P, _P, _I32, _P, _P]),
    "lbm_filter_work_bytes": (_SZ, [_I32, _I32, _I32, ctypes.c_double]),
    "lbm_filter_subsample": (ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_double, _P, _P, _SZ, _P]),
    "lbm_closure_samples": (ctypes.c_int, [_P, _I32, _I32, ctypes.c_double, _I32, _P, _P, _P]),
    "lbm_set_closure_mlp": (ctypes.c_int, [_P, _P]),
    "lbm_closure_correction": (ctypes.c_int, [_P, _P]),
    "lbm_set_correction_interval": (ctypes.c_int, [_P, ctypes.c_int32]),
    "lbm_spectra_bins": (_I32, [_I32]),
    "lbm_spectra_work_bytes": (_SZ, [_I32]),
    "lbm_spectra": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _SZ, _P]),
}

_lib = None


class LbmError(RuntimeError):
    def __init__(self, code: int, func: str, message: str):
        super().__init__(f"{func} failed ({code}): {message}")
        self.code = code


def header_functions() -> list[str]:
    """Names of the functions declared in include/*.h."""
    names = set()
    for path in HEADERS:
        with open(path) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def load():
    """Load liblbmhd.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -m paper_1705_09807_amd.build); there is no fallback path")
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, func: str) -> int:
    if code != LBM_OK:
        msg = _lib.lbm_last_error().decode() if _lib is not None else ""
        raise LbmError(code, func, msg)
    return code
