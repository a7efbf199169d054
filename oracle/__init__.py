"""FP64 CPU oracle for the DeGraF + robust local optical flow path -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this package.
It is a plain, slow, double-precision implementation written from the method's definitions
(DeGraF-Flow, Section 2: "Point detection" with Eq. (1)-(2) and the centroid-selection rule;
"Sparse point tracking" with the robust local flow reading documented in ``degraf_oracle.c``).
It shares no code with the HIP library and never calls it.

The C source is compiled with gcc into ``liboracle.so`` next to this file by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "degraf_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "epic_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ST_CONVERGED, ST_NOT_CONVERGED, ST_ILL_CONDITIONED, ST_OUT_OF_BOUNDS = 0, 1, 2, 3

# Interpolation constants: k neighbours (Section 3 "Parameters"), the flat step cost kappa and
# the weight half-distance h of the geodesic reading (both in edge-map units).
EPIC_DEFAULTS = dict(k=128, kappa=8, h=64)

# Default tracker constants on the 0..255 intensity scale (same meaning as the library's
# default options; the values are restated here, not imported).
DEFAULTS = dict(sigma1=8.0, sigma2=32.0, eps_coarse=1e-2, eps_fine=1e-4, min_eig=1e-4 * 255.0 * 255.0)
# Intensity threshold of the adaptive cross-based supports (grey levels).
CROSS_TAU = 25.0


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99, OpenMP for the loop over points)."""
    if force or _stale():
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, *_SRCS, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _stale() -> bool:
    return not os.path.exists(_LIB_PATH) or any(os.path.getmtime(_LIB_PATH) < os.path.getmtime(f) for f in _SRCS)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _stale():
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.or_detect_count.argtypes = [i32, i32, i32, i32]
    lib.or_detect_count.restype = i64
    lib.or_detect.argtypes = [P, i32, i32, i64, i32, i32, i32, P, P, P, i32]
    lib.or_detect.restype = i64
    lib.or_window_sums.argtypes = [P, i64, i32, i32, i32, i32, i32, P]
    lib.or_window_sums.restype = None
    lib.or_pyr_dims.argtypes = [i32, i32, i32, P]
    lib.or_pyr_dims.restype = None
    lib.or_pyr_down_u8.argtypes = [P, i32, i32, i64, P]
    lib.or_pyr_down_u8.restype = i32
    lib.or_pyr_down_f64.argtypes = [P, i32, i32, P]
    lib.or_pyr_down_f64.restype = i32
    lib.or_bilinear.argtypes = [P, i32, i32, f64, f64]
    lib.or_bilinear.restype = f64
    lib.or_psi.argtypes = [f64, f64, f64]
    lib.or_psi.restype = f64
    lib.or_dpsi.argtypes = [f64, f64, f64]
    lib.or_dpsi.restype = f64
    lib.or_track.argtypes = [P, P, i32, i32, i32, i64, P, i64, i32, i32, i32, f64, f64, f64, f64, f64,
                             i32, i32, f64, i32, P, P, P, P, P, i32]
    lib.or_cross_mask.argtypes = [P, i32, f64, P]
    lib.or_cross_mask.restype = i32
    lib.or_gm_fit.argtypes = [P, P, P, i64, f64, f64, f64, i32, P]
    lib.or_gm_fit.restype = i32
    lib.or_track.restype = i32
    lib.or_track_grad.argtypes = [P, P, i32, i32, P, i64, i32, f64, f64, P, P, P, P, P, P]
    lib.or_track_grad_illum.argtypes = [P, P, i32, i32, P, i64, i32, f64, f64, P, P, P, P, P, P, P]
    lib.or_track_grad_illum.restype = i32
    lib.or_epic_edges.argtypes = [P, i32, i32, i64, P]
    lib.or_epic_edges.restype = None
    lib.or_epic_voronoi.argtypes = [P, i32, i32, i64, P, P, P, i64, i32, P, P, P]
    lib.or_epic_voronoi.restype = i32
    lib.or_epic.argtypes = [P, i32, i32, i64, P, P, P, i64, i32, i32, i32, P, P, P, P, P, P, P]
    lib.or_epic.restype = i32
    lib.or_flow_error.argtypes = [P, P, P, i64, f64, P]
    lib.or_flow_error.restype = None
    lib.or_detect_f64.argtypes = [P, i32, i32, i64, i32, i32, P, P]
    lib.or_detect_f64.restype = i64
    lib.or_detect_grad.argtypes = [P, i32, i32, i64, i32, i32, P, P, P]
    lib.or_detect_grad.restype = i32
    lib.or_track_grad.restype = i32
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def default_threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def detect_count(W: int, H: int, window: int, stride: int) -> int:
    return int(_load().or_detect_count(W, H, window, stride))


def detect(img: np.ndarray, window: int, stride: int, m_mode: int = 0, threads: int | None = None):
    """DeGraF key-points of a uint8 image.  Returns (points[N,2] float64 (x, y), sel[N] uint8,
    response[N] float64)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    N = detect_count(W, H, window, stride)
    pts = np.zeros((N, 2), np.float64)
    sel = np.zeros(N, np.uint8)
    resp = np.zeros(N, np.float64)
    rc = _load().or_detect(_ptr(img), W, H, W, window, stride, m_mode, _ptr(pts), _ptr(sel), _ptr(resp),
                           threads or default_threads())
    if rc < 0:
        raise ValueError(f"or_detect failed: {rc}")
    return pts, sel, resp


def window_sums(img: np.ndarray, x0: int, y0: int, w: int, h: int, m_mode: int = 0):
    """Exact integer sums of one window (Eq. 1-2): (S_pos, sum i*I, sum j*I, S_neg,
    sum i*(1+m-I), sum j*(1+m-I), m), i = row, j = column."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    if not (0 <= x0 and 0 <= y0 and x0 + w <= W and y0 + h <= H):
        raise ValueError("window outside the image")
    out = np.zeros(7, np.int64)
    _load().or_window_sums(_ptr(img), W, x0, y0, w, h, m_mode, _ptr(out))
    return tuple(int(v) for v in out)


def pyr_dims(W: int, H: int, levels: int):
    d = np.zeros(2 * levels, np.int32)
    _load().or_pyr_dims(W, H, levels, _ptr(d))
    return [(int(d[2 * l]), int(d[2 * l + 1])) for l in range(levels)]


def pyramid(img: np.ndarray, levels: int):
    """List of pyramid levels: uint8 in -> uint8 levels; float in -> float64 levels."""
    lib = _load()
    out = []
    if img.dtype == np.uint8:
        cur = np.ascontiguousarray(img)
        out.append(cur)
        for _ in range(levels - 1):
            H, W = cur.shape
            nxt = np.zeros(((H + 1) // 2, (W + 1) // 2), np.uint8)
            if lib.or_pyr_down_u8(_ptr(cur), W, H, W, _ptr(nxt)) != 0:
                raise ValueError("or_pyr_down_u8 failed")
            out.append(nxt)
            cur = nxt
    else:
        cur = np.ascontiguousarray(img, dtype=np.float64)
        out.append(cur)
        for _ in range(levels - 1):
            H, W = cur.shape
            nxt = np.zeros(((H + 1) // 2, (W + 1) // 2), np.float64)
            if lib.or_pyr_down_f64(_ptr(cur), W, H, _ptr(nxt)) != 0:
                raise ValueError("or_pyr_down_f64 failed")
            out.append(nxt)
            cur = nxt
    return out


def bilinear(img: np.ndarray, x: float, y: float) -> float:
    img = np.ascontiguousarray(img, dtype=np.float64)
    H, W = img.shape
    return float(_load().or_bilinear(_ptr(img), W, H, float(x), float(y)))


def psi(r: float, sigma1: float, sigma2: float) -> float:
    return float(_load().or_psi(float(r), float(sigma1), float(sigma2)))


def dpsi(r: float, sigma1: float, sigma2: float) -> float:
    return float(_load().or_dpsi(float(r), float(sigma1), float(sigma2)))


def track(I0: np.ndarray, I1: np.ndarray, points: np.ndarray, levels: int, support: int, iters: int,
          sigma1=DEFAULTS["sigma1"], sigma2=DEFAULTS["sigma2"], eps_coarse=DEFAULTS["eps_coarse"],
          eps_fine=DEFAULTS["eps_fine"], min_eig=DEFAULTS["min_eig"], threads: int | None = None,
          return_iters: bool = False, illum: bool = False, return_illum: bool = False,
          cross: bool = False, tau: float = CROSS_TAU, gm: bool = False, return_gm: bool = False):
    """Track points from I0 to I1.  uint8 images use the uint8 pyramid; anything else is taken
    as real-valued (float64).  ``illum`` selects the gain/offset illumination model, ``cross`` the
    adaptive cross-based supports (threshold ``tau``), ``gm`` the global-motion prior.  Returns
    (flow[n,2] float64, status[n] uint8[, iters[n,L]][, illum[n,2] = (m, c)][, gm model[2,3]])."""
    if I0.shape != I1.shape:
        raise ValueError("I0 and I1 must have the same shape")
    if I0.dtype == np.uint8 and I1.dtype == np.uint8:
        a0, a1, dt = np.ascontiguousarray(I0), np.ascontiguousarray(I1), 0
    else:
        a0 = np.ascontiguousarray(I0, dtype=np.float64)
        a1 = np.ascontiguousarray(I1, dtype=np.float64)
        dt = 1
    H, W = a0.shape
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    flow = np.zeros((n, 2), np.float64)
    st = np.zeros(n, np.uint8)
    its = np.zeros((n, levels), np.int32) if return_iters else None
    mc = np.zeros((n, 2), np.float64) if return_illum else None
    A = np.zeros(6, np.float64)
    rc = _load().or_track(_ptr(a0), _ptr(a1), dt, W, H, W, _ptr(pts), n, levels, support, iters,
                          sigma1, sigma2, eps_coarse, eps_fine, min_eig, int(bool(illum)), int(bool(cross)),
                          float(tau), int(bool(gm)), _ptr(flow), _ptr(st), _ptr(its), _ptr(mc), _ptr(A),
                          threads or default_threads())
    if rc != 0:
        raise ValueError(f"or_track failed: {rc}")
    out = (flow, st)
    if return_iters:
        out += (its,)
    if return_illum:
        out += (mc,)
    if return_gm:
        out += (A.reshape(2, 3),)
    return out


def cross_mask(Tx: np.ndarray, tau: float = None) -> np.ndarray:
    """Adaptive cross-based support of a template given on its (s+2) x (s+2) extension (offsets
    -r-1 .. r+1): uint8 s x s mask, 1 = in the support."""
    Tx = np.ascontiguousarray(Tx, dtype=np.float64)
    e = Tx.shape[0]
    s = e - 2
    assert Tx.shape == (e, e) and s % 2 == 1 and s >= 1
    m = np.zeros((s, s), np.uint8)
    _load().or_cross_mask(_ptr(Tx), s, CROSS_TAU if tau is None else float(tau), _ptr(m))
    return m


def gm_fit(points: np.ndarray, motions: np.ndarray, use: np.ndarray, center, scale: float, iters: int = 10):
    """Robust global affine motion of the samples: (A[2,3], kind) with kind 2 affine, 1
    translation, 0 none; motion ~ A (x - cx, y - cy, 1)."""
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    v = np.ascontiguousarray(motions, dtype=np.float64).reshape(-1, 2)
    u = np.ascontiguousarray(use, dtype=np.uint8).reshape(-1)
    A = np.zeros(6, np.float64)
    kind = _load().or_gm_fit(_ptr(p), _ptr(v), _ptr(u), len(p), float(center[0]), float(center[1]), float(scale),
                             int(iters), _ptr(A))
    return A.reshape(2, 3), int(kind)


def detect_real(img: np.ndarray, window: int, stride: int):
    """The detector on a real-valued image.  Returns (points[N,2] float64, sel[N] uint8)."""
    a = np.ascontiguousarray(img, dtype=np.float64)
    H, W = a.shape
    n = max(detect_count(W, H, window, stride), 0)
    pts = np.zeros((max(n, 1), 2), np.float64)
    sel = np.zeros(max(n, 1), np.uint8)
    rc = _load().or_detect_f64(_ptr(a), W, H, W, window, stride, _ptr(pts), _ptr(sel))
    if rc < 0:
        raise ValueError(f"or_detect_f64 failed: {rc}")
    return pts[:n], sel[:n]


def detect_grad(img: np.ndarray, window: int, stride: int, sel: np.ndarray, dpoints: np.ndarray) -> np.ndarray:
    """dL/dI of the detected points for upstream gradient dpoints = dL/dp (real-valued image)."""
    a = np.ascontiguousarray(img, dtype=np.float64)
    H, W = a.shape
    s = np.ascontiguousarray(sel, dtype=np.uint8)
    d = np.ascontiguousarray(dpoints, dtype=np.float64).reshape(-1, 2)
    dI = np.zeros((H, W), np.float64)
    rc = _load().or_detect_grad(_ptr(a), W, H, W, window, stride, _ptr(s), _ptr(d), _ptr(dI))
    if rc != 0:
        raise ValueError(f"or_detect_grad failed: {rc}")
    return dI


def track_grad(I0: np.ndarray, I1: np.ndarray, points: np.ndarray, support: int, flow: np.ndarray,
               status: np.ndarray, dflow: np.ndarray, sigma1=DEFAULTS["sigma1"], sigma2=DEFAULTS["sigma2"],
               return_dpoints: bool = False):
    """Implicit gradient (dL/dI0, dL/dI1[, dL/dp]) at the converged level-0 fixed point, for
    upstream gradient dflow = dL/du (points with status != CONVERGED contribute nothing)."""
    a0 = np.ascontiguousarray(I0, dtype=np.float64)
    a1 = np.ascontiguousarray(I1, dtype=np.float64)
    H, W = a0.shape
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    fl = np.ascontiguousarray(flow, dtype=np.float64).reshape(-1, 2)
    st = np.ascontiguousarray(status, dtype=np.uint8)
    df = np.ascontiguousarray(dflow, dtype=np.float64).reshape(-1, 2)
    dI0 = np.zeros((H, W), np.float64)
    dI1 = np.zeros((H, W), np.float64)
    dp = np.zeros((pts.shape[0], 2), np.float64) if return_dpoints else None
    rc = _load().or_track_grad(_ptr(a0), _ptr(a1), W, H, _ptr(pts), pts.shape[0], support, sigma1, sigma2,
                               _ptr(fl), _ptr(st), _ptr(df), _ptr(dI0), _ptr(dI1), _ptr(dp))
    if rc != 0:
        raise ValueError(f"or_track_grad failed: {rc}")
    if return_dpoints:
        return dI0, dI1, dp
    return dI0, dI1


def track_grad_illum(I0: np.ndarray, I1: np.ndarray, points: np.ndarray, support: int, flow: np.ndarray,
                     illum: np.ndarray, status: np.ndarray, dflow: np.ndarray, sigma1=DEFAULTS["sigma1"],
                     sigma2=DEFAULTS["sigma2"], return_dpoints: bool = False):
    """Implicit gradient (dL/dI0, dL/dI1) of the illumination-model tracker at its converged
    level-0 fixed point (flow and illum = (m, c) as the forward pass returned them), and with
    ``return_dpoints`` also dL/dp w.r.t. the point positions."""
    a0 = np.ascontiguousarray(I0, dtype=np.float64)
    a1 = np.ascontiguousarray(I1, dtype=np.float64)
    H, W = a0.shape
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    fl = np.ascontiguousarray(flow, dtype=np.float64).reshape(-1, 2)
    mc = np.ascontiguousarray(illum, dtype=np.float64).reshape(-1, 2)
    st = np.ascontiguousarray(status, dtype=np.uint8)
    df = np.ascontiguousarray(dflow, dtype=np.float64).reshape(-1, 2)
    dI0 = np.zeros((H, W), np.float64)
    dI1 = np.zeros((H, W), np.float64)
    dp = np.zeros((pts.shape[0], 2), np.float64) if return_dpoints else None
    rc = _load().or_track_grad_illum(_ptr(a0), _ptr(a1), W, H, _ptr(pts), pts.shape[0], support, sigma1, sigma2,
                                     _ptr(fl), _ptr(mc), _ptr(st), _ptr(df), _ptr(dI0), _ptr(dI1), _ptr(dp))
    if rc != 0:
        raise ValueError(f"or_track_grad_illum failed: {rc}")
    if return_dpoints:
        return dI0, dI1, dp
    return dI0, dI1


# ---- dense interpolation (Section 2 "Interpolation") ------------------------------------------

def epic_edges(I: np.ndarray) -> np.ndarray:
    """Integer edge map |I(x+1)-I(x-1)| + |I(y+1)-I(y-1)| of a uint8 frame (replicated border)."""
    a = np.ascontiguousarray(I, dtype=np.uint8)
    H, W = a.shape
    E = np.zeros((H, W), np.int32)
    _load().or_epic_edges(_ptr(a), W, H, W, _ptr(E))
    return E


def epic_voronoi(I: np.ndarray, points: np.ndarray, status: np.ndarray, kappa=EPIC_DEFAULTS["kappa"]):
    """Geodesic Voronoi partition of the pixels among the converged points: (D int64 [H, W],
    L int32 [H, W], alive uint8 [n])."""
    a = np.ascontiguousarray(I, dtype=np.uint8)
    H, W = a.shape
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    st = np.ascontiguousarray(status, dtype=np.uint8)
    D = np.zeros((H, W), np.int64)
    L = np.zeros((H, W), np.int32)
    alive = np.zeros(pts.shape[0], np.uint8)
    rc = _load().or_epic_voronoi(_ptr(a), W, H, W, _ptr(pts), None, _ptr(st), pts.shape[0], kappa, _ptr(D),
                                 _ptr(L), _ptr(alive))
    if rc != 0:
        raise ValueError(f"or_epic_voronoi failed: {rc}")
    return D, L, alive


def epic(I: np.ndarray, points: np.ndarray, flow: np.ndarray, status: np.ndarray, k=EPIC_DEFAULTS["k"],
         kappa=EPIC_DEFAULTS["kappa"], h=EPIC_DEFAULTS["h"], full: bool = False):
    """Dense flow float64 [H, W, 2] interpolated from the converged points.  With ``full`` also
    returns a dict of the intermediate results: D, L, nb [n, k], nd [n, k], model [n, 6], alive."""
    a = np.ascontiguousarray(I, dtype=np.uint8)
    H, W = a.shape
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 2)
    fl = np.ascontiguousarray(flow, dtype=np.float64).reshape(-1, 2)
    st = np.ascontiguousarray(status, dtype=np.uint8)
    n = pts.shape[0]
    dense = np.zeros((H, W, 2), np.float64)
    D = np.zeros((H, W), np.int64) if full else None
    L = np.zeros((H, W), np.int32) if full else None
    nb = np.zeros((n, k), np.int32) if full else None
    nd = np.zeros((n, k), np.int64) if full else None
    model = np.zeros((n, 6), np.float64) if full else None
    alive = np.zeros(n, np.uint8) if full else None
    rc = _load().or_epic(_ptr(a), W, H, W, _ptr(pts), _ptr(fl), _ptr(st), n, k, kappa, h, _ptr(dense), _ptr(D),
                         _ptr(L), _ptr(nb), _ptr(nd), _ptr(model), _ptr(alive))
    if rc != 0:
        raise ValueError(f"or_epic failed: {rc}")
    if full:
        return dense, dict(D=D, L=L, nb=nb, nd=nd, model=model, alive=alive)
    return dense


def flow_error(flow: np.ndarray, ref: np.ndarray, valid: np.ndarray | None = None, thresh: float = 3.0):
    """(mean endpoint error, fraction of pixels with error > thresh px, pixel count) over ``valid``."""
    f = np.ascontiguousarray(flow, dtype=np.float64).reshape(-1, 2)
    r = np.ascontiguousarray(ref, dtype=np.float64).reshape(-1, 2)
    v = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8).reshape(-1)
    out = np.zeros(3, np.float64)
    _load().or_flow_error(_ptr(f), _ptr(r), _ptr(v), f.shape[0], thresh, _ptr(out))
    cnt = out[2]
    return (out[0] / cnt if cnt else float("nan")), (out[1] / cnt if cnt else float("nan")), int(cnt)
