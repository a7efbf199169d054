"""ctypes loader for ``libdegraf_flow.so`` (the gfx950 HIP library) -- argument marshalling only.

The library must have been built (``paper_1901_09971_amd/build.py`` or ``__graft_entry__.build``).
There is no fallback: if the shared object is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdegraf_flow.so")

DGF_OK = 0
DGF_U8, DGF_F32 = 0, 1
DGF_TRACK_ILLUM = 1
DGF_TRACK_CROSS = 2
DGF_TRACK_GLOBAL = 4
DGF_MAX_LEVELS = 12
DGF_ERR_SCRATCH = -6
DGF_TRACK_STATIC_MAX_BYTES = 16 << 20
ST_CONVERGED, ST_NOT_CONVERGED, ST_ILL_CONDITIONED, ST_OUT_OF_BOUNDS = 0, 1, 2, 3


class DgfImage(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch_bytes", ctypes.c_int64), ("dtype", ctypes.c_int32)]


class DgfTrackOpts(ctypes.Structure):
    _fields_ = [("sigma1", ctypes.c_float), ("sigma2", ctypes.c_float), ("eps_coarse", ctypes.c_float),
                ("eps_fine", ctypes.c_float), ("min_eig", ctypes.c_float), ("flags", ctypes.c_int32),
                ("cross_tau", ctypes.c_float)]


class DgfPairDesc(ctypes.Structure):
    _fields_ = [("I0", DgfImage), ("I1", DgfImage), ("window", ctypes.c_int32), ("stride", ctypes.c_int32)]


class DgfTuning(ctypes.Structure):
    _fields_ = [("lanes_per_point", ctypes.c_int32), ("waves_per_group", ctypes.c_int32), ("margin", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("ms", ctypes.c_float)]


class DgfEpicOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("kappa", ctypes.c_int32), ("half_dist", ctypes.c_int32)]


class DgfError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


_lib = None

# every exported symbol with (restype, argtypes); the header declares exactly these
P, I32, I64, SZ, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
IMG = ctypes.POINTER(DgfImage)
OPTS = ctypes.POINTER(DgfTrackOpts)
SIGNATURES = {
    "dgf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dgf_version": (ctypes.c_int, []),
    "dgf_track_opts_default": (ctypes.c_int, [OPTS]),
    "dgf_detect_count": (I64, [I32, I32, I32, I32]),
    "dgf_detect": (ctypes.c_int, [IMG, I32, I32, P, P, P, I64, P]),
    "dgf_pyramid_layout": (SZ, [I32, I32, I32, I32, P, P]),
    "dgf_pyramid": (ctypes.c_int, [IMG, I32, P, SZ, P]),
    "dgf_track_workspace_bytes": (SZ, [I32, I32, I32, I32]),
    "dgf_gm_workspace_bytes": (SZ, []),
    "dgf_gm_fit": (ctypes.c_int, [P, P, P, I64, I32, I32, ctypes.c_double, P, SZ, P, P]),
    "dgf_track": (ctypes.c_int, [IMG, IMG, P, I64, I32, I32, I32, OPTS, P, SZ, P, P, P, P, P]),
    "dgf_track_static": (ctypes.c_int, [IMG, IMG, P, I64, I32, I32, I32, OPTS, P, P, P, P, P]),
    "dgf_track_pyramids": (ctypes.c_int, [IMG, IMG, I32, P, SZ, P]),
    "dgf_track_run": (ctypes.c_int, [IMG, IMG, P, I64, I32, I32, I32, OPTS, P, SZ, P, P, P, P, P]),
    "dgf_detect_pyramids": (ctypes.c_int, [IMG, IMG, I32, I32, I32, P, SZ, P, P, P, I64, P]),
    "dgf_track_backward": (ctypes.c_int, [IMG, IMG, P, I64, I32, OPTS, P, P, P, P, P, P, P, P]),
    "dgf_detect_backward": (ctypes.c_int, [IMG, I32, I32, P, P, I64, P, I64, P]),
    "dgf_batch_create": (ctypes.c_int, [ctypes.POINTER(DgfPairDesc), I32, I32, I32, I32, OPTS,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "dgf_batch_num_points": (I64, [P]),
    "dgf_batch_point_offsets": (ctypes.c_int, [P, P]),
    "dgf_batch_run": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "dgf_batch_front": (ctypes.c_int, [P, P, P]),
    "dgf_batch_track": (ctypes.c_int, [P, P, P, P, P, P, P]),
    "dgf_batch_capture": (ctypes.c_int, [P, P, P, P, P, P]),
    "dgf_batch_replay": (ctypes.c_int, [P, P]),
    "dgf_batch_level": (ctypes.c_int, [P, I32, I32, I32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(I64),
                                       ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "dgf_batch_grad_size": (I64, [P, P]),
    "dgf_batch_backward": (ctypes.c_int, [P, P, P, P, P, P, P, P]),
    "dgf_batch_destroy": (ctypes.c_int, [P]),
    "dgf_epic_opts_default": (ctypes.c_int, [ctypes.POINTER(DgfEpicOpts)]),
    "dgf_epic_workspace_bytes": (SZ, [I32, I32, I64]),
    "dgf_epic": (ctypes.c_int, [IMG, P, P, P, I64, ctypes.POINTER(DgfEpicOpts), P, SZ, P, I64, P, P, P, P, P, P]),
    "dgf_epic_async": (ctypes.c_int, [IMG, P, P, P, I64, ctypes.POINTER(DgfEpicOpts), P, SZ, P, I64, P, P, P, P, P, I32,
                                      P, P]),
    "dgf_get_tuning": (ctypes.c_int, [I32, I32, I32, I64, ctypes.POINTER(DgfTuning)]),
    "dgf_set_tuning": (ctypes.c_int, [I32, I32, ctypes.POINTER(DgfTuning)]),
    "dgf_autotune": (ctypes.c_int, [IMG, IMG, P, I64, I32, I32, I32, OPTS, P, SZ, P, P, ctypes.c_char_p,
                                    ctypes.POINTER(DgfTuning), P]),
}


def lib():
    """The loaded library; raises if it is not built.  Never falls back to anything else."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run paper_1901_09971_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().dgf_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library itself is missing
        return f"error {code}"


def check(code: int, where: str) -> None:
    if code != DGF_OK:
        raise DgfError(code, where)
