"""ctypes binding of libprism.so (the C ABI in include/prism.h).

Argument marshalling only: every step of the pass runs in the library's HIP
kernels.  Loading fails loudly if the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprism.so")

PRISM_OK = 0
PRISM_E_INVALID = -1
PRISM_E_UNSUPPORTED = -2
PRISM_E_HIP = -3
PRISM_E_WORKSPACE = -4
PRISM_E_ALLOC = -5
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "UNSUPPORTED", -3: "HIP", -4: "WORKSPACE", -5: "ALLOC"}

MSE, RICIAN = 0, 1
BIAS = {"none": 0, "poly2": 1, "trilinear8": 2}
PRIOR_BITS = {"spatial": 1, "rep": 2, "sparse": 4, "cal": 8, "orphan": 16, "continuity": 32,
              "ordering": 64, "tv": 128}
ST_NONFINITE_LOSS, ST_NONFINITE_GRAD, ST_ZERO_DIRECTION = 1, 2, 4
LOSS_TERMS = ("data", "spatial", "rep", "sparse", "orphan", "continuity", "ordering", "cal", "tv", "total")
LOSS_TOTAL = 9
MAX_K = 6
MAX_MEAS = 1024
NOALLOC_WORKSPACE_BYTES = 64 << 20


class PrismError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libprism {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Acq(ctypes.Structure):
    _fields_ = [("n_meas", ctypes.c_int32), ("bval", ctypes.POINTER(ctypes.c_float)),
                ("bvec", ctypes.POINTER(ctypes.c_float))]


class GroupDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("K", ctypes.c_int32), ("mode", ctypes.c_int32), ("bias", ctypes.c_int32),
                ("acq", ctypes.c_int32), ("neighbourhood", ctypes.c_int32),
                ("learn_diffusivity", ctypes.c_int32), ("priors", ctypes.c_uint32),
                ("mask", ctypes.POINTER(ctypes.c_uint8))]


class Model(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in (
        "d_csf", "d_gm", "d_res", "d_par", "d_perp", "lam_sp", "huber_delta", "lam_rep",
        "lam_sparse", "tau_sparse", "lam_alpha", "lam_beta", "lam_bias", "lam_orphan", "s0_orphan",
        "lam_cont", "lam_order", "lam_tv")]


class GroupInfo(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int64), ("n_meas", ctypes.c_int32), ("K", ctypes.c_int32),
                ("n_params_vox", ctypes.c_int32), ("n_bias", ctypes.c_int32),
                ("n_cal", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("micro_offset", ctypes.c_int64), ("cal_offset", ctypes.c_int64),
                ("y_offset", ctypes.c_int64)]


class ProblemInfo(ctypes.Structure):
    _fields_ = [("n_vox", ctypes.c_int64), ("n_micro", ctypes.c_int64), ("n_cal", ctypes.c_int64),
                ("n_y", ctypes.c_int64), ("n_groups", ctypes.c_int32), ("n_buckets", ctypes.c_int32)]


class Launch(ctypes.Structure):
    _fields_ = [("vox_per_lane", ctypes.c_int32), ("n_split", ctypes.c_int32),
                ("item_vox", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("stagger", ctypes.c_int32), ("concurrent", ctypes.c_int32)]


class BucketLaunch(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_meas", "K", "mode", "learn_diffusivity", "vox_per_lane",
                                               "n_split", "item_vox")]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F = ctypes.c_float

SIGNATURES = {
    "prism_abi_version": (_I32, []),
    "prism_last_error": (ctypes.c_char_p, []),
    "prism_model_defaults": (None, [ctypes.POINTER(Model)]),
    "prism_problem_create": (_I32, [ctypes.POINTER(_P), ctypes.POINTER(GroupDesc), _I32,
                                    ctypes.POINTER(Acq), _I32, ctypes.POINTER(Model)]),
    "prism_problem_destroy": (_I32, [_P]),
    "prism_problem_info": (_I32, [_P, ctypes.POINTER(ProblemInfo)]),
    "prism_group_info": (_I32, [_P, _I32, ctypes.POINTER(GroupInfo)]),
    "prism_problem_tune": (_I32, [_P, ctypes.POINTER(Launch)]),
    "prism_problem_launch": (_I32, [_P, ctypes.POINTER(Launch)]),
    "prism_problem_tune_buckets": (_I32, [_P, ctypes.POINTER(Launch), ctypes.POINTER(BucketLaunch), _I32]),
    "prism_problem_buckets": (_I32, [_P, ctypes.POINTER(BucketLaunch), _I32, ctypes.POINTER(_I32)]),
    "prism_problem_plan_info": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "prism_build_id": (ctypes.c_char_p, []),
    "prism_workspace_bytes": (_I32, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "prism_synthesize": (_I32, [_P, _P, _P, _P, _P]),
    "prism_loss_grad": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "prism_loss_grad_noalloc": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "prism_adam_step": (_I32, [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _P, _P]),
    "prism_rprop_step": (_I32, [_P, _P, _P, _P, _I64, _F, _F, _F, _F, _P]),
    "prism_iteration_adam": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _F, _F, _F, _F, _I32, _P, _P, _I32,
                                    _P, _P, _P, ctypes.c_size_t, _P, _P]),
    "prism_rician_terms": (_I32, [_P, _P, _P, _P, _I64, _P]),
    "prism_stitch_plan": (_I32, [_P, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "prism_stitch_maps": (_I32, [_P, _P, _P, _P]),
    "prism_profile_enable": (_I32, [_P, _I32, _I32]),
    "prism_profile_read": (_I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I32)]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_00250_amd.build` "
                              "(the HIP library is required; there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != PRISM_OK:
        raise PrismError(code, lib().prism_last_error().decode(errors="replace"))


def model_defaults() -> Model:
    m = Model()
    lib().prism_model_defaults(ctypes.byref(m))
    return m
