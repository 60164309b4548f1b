"""ctypes binding of librdseg.so (C ABI in include/rdseg.h).

Argument marshalling only: every step of the method runs in the HIP library.
If the library has not been built this module raises instead of falling back
to anything else.
"""
import atexit
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# RDSEG_LIBRARY selects another build of the same ABI (the sanitizer build)
LIB_PATH = os.environ.get("RDSEG_LIBRARY") or os.path.join(HERE, "librdseg.so")

RDSEG_OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "invalid shape", 3: "workspace too small",
                4: "HIP error", 5: "tape missing or inconsistent",
                6: "a bounded on-chip wait expired"}
RDSEG_ERR_TIMEOUT = 6


class RdsegError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"rdseg status {status} ({STATUS_NAMES.get(status, '?')}): {message}")
        self.status = status


class Shape(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("ld", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("theta", ctypes.c_double),
                ("tau", ctypes.c_double), ("delta", ctypes.c_double),
                ("iters", ctypes.c_int32), ("iters_per_launch", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("components", ctypes.c_int32), ("resident", ctypes.c_int32)]


class Shape3(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("ld", ctypes.c_int64), ("lds", ctypes.c_int64)]


class PdParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("tau", ctypes.c_double),
                ("sigma", ctypes.c_double), ("delta", ctypes.c_double),
                ("iters", ctypes.c_int32), ("iters_per_launch", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


class Fit(ctypes.Structure):
    _fields_ = [("z", ctypes.c_void_p), ("P", ctypes.c_void_p), ("c1", ctypes.c_double),
                ("c2", ctypes.c_double), ("gamma", ctypes.c_double)]


class Image(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("s", Shape), ("lambda_", ctypes.c_double),
                ("delta", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t
_d = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "rdseg_workspace_size": (_sz, [ctypes.POINTER(Shape), ctypes.POINTER(Params)]),
    "rdseg_tape_size": (_sz, [ctypes.POINTER(Shape), ctypes.POINTER(Params)]),
    "rdseg_backward_workspace_size": (_sz, [ctypes.POINTER(Shape), ctypes.POINTER(Params)]),
    "rdseg_active_set": (ctypes.c_int, [_vp, Shape, _d, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "rdseg_band_workspace_size": (_sz, []),
    "rdseg_band_threshold": (ctypes.c_int, [_vp, Shape, _d, _vp, _vp, _sz, _vp]),
    "rdseg_solve": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp, _sz, _vp]),
    "rdseg_pd_workspace_size": (_sz, [ctypes.POINTER(Shape)]),
    "rdseg_solve_pd": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(PdParams), _vp, _vp, _vp, _vp,
                                      _vp, _sz, _vp]),
    "rdseg_workspace_size3": (_sz, [ctypes.POINTER(Shape3)]),
    "rdseg_solve3d": (ctypes.c_int, [_vp, Shape3, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp,
                                     _vp, _sz, _vp]),
    "rdseg_metrics_workspace_size": (_sz, []),
    "rdseg_metrics": (ctypes.c_int, [_vp, _vp, Shape, _d, _vp, _vp, _sz, _vp]),
    "rdseg_solve_until": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(Params), _d, ctypes.c_int32,
                                         ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _sz, _vp]),
    "rdseg_batched_workspace_size": (_sz, [ctypes.POINTER(Image), _i32, _i32, _i32]),
    "rdseg_solve_batched": (ctypes.c_int, [ctypes.POINTER(Image), _i32, _d, _d, _i32, _i32, _i32,
                                           _i32, ctypes.POINTER(_vp), _vp, _sz, _vp]),
    "rdseg_plan_destroy": (ctypes.c_int, [_vp]),
    "rdseg_autotune_batched": (ctypes.c_int, [ctypes.POINTER(Image), _i32, _d, _d, _i32, _i32,
                                              _i32, _i32, _i32, _vp, _sz, _vp,
                                              ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                              ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "rdseg_batched_lookup": (ctypes.c_int, [ctypes.POINTER(Image), _i32, _d,
                                            ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                            ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                            ctypes.POINTER(_i32)]),
    "rdseg_backward": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp,
                                      ctypes.POINTER(Fit), _vp, _vp, _vp, _vp, _sz, _vp]),
    "rdseg_fit_forward": (ctypes.c_int, [ctypes.POINTER(Fit), Shape, _vp, _vp]),
    "rdseg_reduce_workspace_size": (_sz, [ctypes.POINTER(Shape)]),
    "rdseg_fit_backward": (ctypes.c_int, [ctypes.POINTER(Fit), Shape, _vp, _vp, _vp, _vp, _vp, _sz,
                                          _vp]),
    "rdseg_autotune": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(Params), _i32, _vp, _vp, _vp, _vp,
                                      _sz, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32)]),
    "rdseg_config_count": (_i32, []),
    "rdseg_config_get": (ctypes.c_int, [_i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                        ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "rdseg_timing_enable": (ctypes.c_int, [_i32]),
    "rdseg_timing_read": (ctypes.c_int, [_i32, ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(_d), ctypes.POINTER(ctypes.c_int64)]),
    "rdseg_timing_read_form": (ctypes.c_int, [_i32, _i32, ctypes.POINTER(_d),
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_d),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "rdseg_timing_reset": (ctypes.c_int, []),
    "rdseg_set_resident": (ctypes.c_int, [_i32]),
    "rdseg_set_components": (ctypes.c_int, [_i32]),
    "rdseg_set_batched_form": (ctypes.c_int, [_i32]),
    "rdseg_set_adjoint_form": (ctypes.c_int, [_i32, _i32]),
    "rdseg_tune_cache_export": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "rdseg_tune_cache_import": (ctypes.c_int, [ctypes.c_char_p]),
    "rdseg_tune_lookup": (ctypes.c_int, [ctypes.POINTER(Shape), _d, ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32)]),
    "rdseg_tune_cache_clear": (ctypes.c_int, []),
    "rdseg_solve_status": (ctypes.c_int, [ctypes.POINTER(Shape), _vp, _sz, _vp]),
    "rdseg_solve_noalloc": (ctypes.c_int, [_vp, Shape, ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                                           _vp, _vp]),
    "rdseg_set_resident_wait": (ctypes.c_int, [ctypes.c_int64]),
    "rdseg_release": (ctypes.c_int, []),
    "rdseg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rdseg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load librdseg.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with "
                           "`python -m paper_1807_11534_amd.build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    # release the library's streams, events and pinned buffers while the HIP
    # runtime is still up (interpreter exit runs before the runtime's teardown)
    atexit.register(_release)
    return lib


def _release():
    if _lib is not None:
        _lib.rdseg_release()


def check(status):
    if status != RDSEG_OK:
        msg = load().rdseg_last_error()
        raise RdsegError(status, msg.decode() if msg else "")
