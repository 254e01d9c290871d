"""ctypes loader for the HIP library ``liblhdm.so`` (C ABI in ``include/lhdm.h``).

Loading fails loudly when the library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblhdm.so")

LHDM_EINVAL = -1
LHDM_EWORKSPACE = -2
LHDM_EHIP = -3
LHDM_EUNSUPPORTED = -4

STATUS_OK = 0
STATUS_MAXITER = 1
STATUS_NONFINITE = 2
STATUS_RANK = 3


class LhdmParams(ctypes.Structure):
    _fields_ = [
        ("tau1", ctypes.c_double),
        ("tau2", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("kkt_tol", ctypes.c_double),
        ("kmax", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("max_inner", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class LhdmInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32),
        ("inner_iters", ctypes.c_int32),
        ("jloop_drops", ctypes.c_int32),
        ("n_passive", ctypes.c_int32),
        ("cq_panels", ctypes.c_int32),
        ("kkt_residual", ctypes.c_double),
        ("objective", ctypes.c_double),
    ]


INFO_BYTES = ctypes.sizeof(LhdmInfo)

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_dbl = ctypes.c_double
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)

SIGNATURES = {
    "lhdm_default_params": (None, [ctypes.POINTER(LhdmParams)]),
    "lhdm_workspace_bytes": (_sz, [_i32, _i32, ctypes.POINTER(LhdmParams)]),
    "lhdm_solve": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp, ctypes.POINTER(LhdmParams),
                                  _vp, _vp, _vp, _vp, _vp, _sz]),
    "lh_solve": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _sz]),
    "lhdm_signed_workspace_bytes": (_sz, [_i32, _i32, ctypes.POINTER(LhdmParams)]),
    "lhdm_l1_workspace_bytes": (_sz, [_i32, _i32, ctypes.POINTER(LhdmParams)]),
    "lhdm_solve_l1": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp, _dbl, ctypes.POINTER(LhdmParams), _vp, _vp,
                                     _vp, _vp, _vp, _sz]),
    "lhdm_solve_signed": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp, ctypes.POINTER(LhdmParams), _i32, _vp, _vp,
                                         _vp, _vp, _vp, _sz]),
    "lhdm_batched_workspace_bytes": (_sz, [_i32, _pi32, _pi32, ctypes.POINTER(LhdmParams)]),
    "lhdm_solve_batched": (ctypes.c_int, [_vp, _i32, _pi32, _pi32, _pi64, _vp, _pi64, _vp, _pi64, _vp, _vp,
                                          ctypes.POINTER(LhdmParams), _i32, _vp, _vp, _sz]),
    "lhdm_solve_batched_noalloc": (ctypes.c_int, [_vp, _i32, _pi32, _pi32, _pi64, _vp, _pi64, _vp, _pi64, _vp,
                                                  _vp, ctypes.POINTER(LhdmParams), _i32, _vp]),
    "lhdm_backward_workspace_bytes": (_sz, [_i32, _pi32, _pi32]),
    "lhdm_backward": (ctypes.c_int, [_vp, _i32, _pi32, _pi32, _pi64, _vp, _pi64, _vp, _pi64, _vp, _vp, _vp,
                                     _vp, _vp, _vp, _sz]),
    "lhdm_profile_enable": (None, [ctypes.c_int]),
    "lhdm_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)]),
    "lhdm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lhdm_last_hip_error": (ctypes.c_int, []),
    "lhdm_release": (None, []),
    # test-only entry points (include/lhdm_testing.h)
    "lhdm_test_downdate": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _i32, _pi32, _vp, _vp, _vp, _pi32,
                                          _pi32]),
    "lhdm_test_trsv": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _pi32]),
    "lhdm_test_cq_factors": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                            ctypes.POINTER(ctypes.c_double)]),
}

_LIB = None


def load():
    """Load ``liblhdm.so`` (raises if it is missing: build it with ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class LhdmError(RuntimeError):
    pass


def check(rc: int) -> None:
    if rc == 0:
        return
    lib = load()
    msg = lib.lhdm_status_string(rc).decode()
    if rc == LHDM_EHIP:
        msg += f" (hipError {lib.lhdm_last_hip_error()})"
    raise LhdmError(f"lhdm call failed: {rc}: {msg}")
