"""Independent brute-force references used to pin the FP64 oracle (CPU only).

Nothing here is shared with the oracle or with the HIP library:

* ``degraf_window_exact``: Eq. (1)-(2) and the selection rule of DeGraF-Flow (Section 2, "Point
  detection") in exact rational arithmetic (``fractions.Fraction``), for tiny windows.
* ``pyr_down_scipy``: one pyramid reduction built from ``scipy.ndimage.correlate1d`` with the
  binomial kernel [1, 4, 6, 4, 1] and replicated borders (``mode='nearest'``).
* ``lk_pyramidal``: textbook least-squares pyramidal Lucas-Kanade (the limit of the robust
  tracker when both robust thresholds are infinite), vectorised over points, using
  ``scipy.ndimage.map_coordinates(order=1, mode='nearest')`` for bilinear sampling; the template
  gradient is the central difference of the sampled image at +-1 px.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy import ndimage


def degraf_window_exact(win, m_mode: int = 0):
    """win: list of rows of ints.  Returns dict with exact S_pos, S_neg, C_pos=(col, row),
    C_neg=(col, row) as Fractions, and the selected point offset and flag."""
    h = len(win)
    w = len(win[0])
    m = max(max(r) for r in win) if m_mode == 0 else 255
    sp = sum(win[i][j] for i in range(h) for j in range(w))
    sn = sum(1 + m - win[i][j] for i in range(h) for j in range(w))
    cp = None
    if sp > 0:
        cp = (Fraction(sum(j * win[i][j] for i in range(h) for j in range(w)), sp),
              Fraction(sum(i * win[i][j] for i in range(h) for j in range(w)), sp))
    cn = (Fraction(sum(j * (1 + m - win[i][j]) for i in range(h) for j in range(w)), sn),
          Fraction(sum(i * (1 + m - win[i][j]) for i in range(h) for j in range(w)), sn))
    neg = sn > sp
    return dict(S_pos=sp, S_neg=sn, C_pos=cp, C_neg=cn, neg=neg, point=cn if neg else cp, m=m)


def pyr_down_scipy(img: np.ndarray) -> np.ndarray:
    """One level down: binomial 5-tap on both axes, replicated border, keep even pixels.
    uint8 -> uint8 with round-half-up of the exact integer sum / 256; float -> float64 exact."""
    k = np.array([1, 4, 6, 4, 1])
    if img.dtype == np.uint8:
        a = img.astype(np.int64)
        a = ndimage.correlate1d(a, k, axis=1, mode="nearest")
        a = ndimage.correlate1d(a, k, axis=0, mode="nearest")
        return ((a[::2, ::2] + 128) // 256).astype(np.uint8)
    a = img.astype(np.float64)
    a = ndimage.correlate1d(a, k / 16.0, axis=1, mode="nearest")
    a = ndimage.correlate1d(a, k / 16.0, axis=0, mode="nearest")
    return a[::2, ::2]


def _sample(img, xs, ys):
    return ndimage.map_coordinates(img, [ys.ravel(), xs.ravel()], order=1, mode="nearest").reshape(xs.shape)


def lk_pyramidal(I0, I1, pts, levels, support, iters, eps_coarse, eps_fine):
    """Least-squares pyramidal LK: per level, template at p/2^l + k, Gauss-Newton with the
    template gradient, stop when the step norm drops below eps, propagate 2 (g + d).
    Returns (flow[n,2], converged_at_level0[n] bool)."""
    P0, P1 = [I0], [I1]
    for _ in range(levels - 1):
        P0.append(pyr_down_scipy(P0[-1]))
        P1.append(pyr_down_scipy(P1[-1]))
    P0 = [p.astype(np.float64) for p in P0]
    P1 = [p.astype(np.float64) for p in P1]
    pts = np.asarray(pts, np.float64)
    n = len(pts)
    r = support // 2
    ky, kx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    kx, ky = kx.ravel()[None, :], ky.ravel()[None, :]
    g = np.zeros((n, 2))
    d = np.zeros((n, 2))
    conv = np.zeros(n, bool)
    for l in range(levels - 1, -1, -1):
        pl = pts / 2.0 ** l
        X, Y = pl[:, :1] + kx, pl[:, 1:] + ky
        T = _sample(P0[l], X, Y)
        GX = 0.5 * (_sample(P0[l], X + 1.0, Y) - _sample(P0[l], X - 1.0, Y))
        GY = 0.5 * (_sample(P0[l], X, Y + 1.0) - _sample(P0[l], X, Y - 1.0))
        a, b, c = (GX * GX).sum(1), (GX * GY).sum(1), (GY * GY).sum(1)
        det = a * c - b * b
        d = np.zeros((n, 2))
        active = np.ones(n, bool)
        conv = np.zeros(n, bool)
        eps = eps_coarse if l > 0 else eps_fine
        for _ in range(iters):
            if not active.any():
                break
            J = _sample(P1[l], X + (g[:, :1] + d[:, :1]), Y + (g[:, 1:] + d[:, 1:]))
            res = J - T
            bx, by = -(res * GX).sum(1), -(res * GY).sum(1)
            sx = (c * bx - b * by) / det
            sy = (a * by - b * bx) / det
            d[active, 0] += sx[active]
            d[active, 1] += sy[active]
            done = active & (np.hypot(sx, sy) < eps)
            conv |= done
            active &= ~done
        if l > 0:
            g = 2.0 * (g + d)
    return g + d, conv


def min_eig_per_level(I0, pts, levels, support):
    """lambda_min of the template-gradient matrix G0 = sum g g^T divided by support^2, per point and
    level (central differences at +-1 px of the bilinear interpolant).  Returns [n][levels]."""
    P0 = [I0]
    for _ in range(levels - 1):
        P0.append(pyr_down_scipy(P0[-1]))
    P0 = [p.astype(np.float64) for p in P0]
    pts = np.asarray(pts, np.float64)
    r = support // 2
    ky, kx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    kx, ky = kx.ravel()[None, :], ky.ravel()[None, :]
    out = np.zeros((len(pts), levels))
    for l in range(levels):
        pl = pts / 2.0 ** l
        X, Y = pl[:, :1] + kx, pl[:, 1:] + ky
        GX = 0.5 * (_sample(P0[l], X + 1.0, Y) - _sample(P0[l], X - 1.0, Y))
        GY = 0.5 * (_sample(P0[l], X, Y + 1.0) - _sample(P0[l], X, Y - 1.0))
        a, b, c = (GX * GX).sum(1), (GX * GY).sum(1), (GY * GY).sum(1)
        out[:, l] = (0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + b * b)) / support ** 2
    return out


def lk_pyramidal_illum(I0, I1, pts, levels, support, iters, eps_coarse, eps_fine):
    """Least-squares pyramidal LK with a per-point gain and offset, I1(p + k + u) ~ (1 + m) T_k + c:
    per level, Gauss-Newton on (d, m, c) with residual derivatives ((1 + m) g, -T, -1), solved as a
    4 x 4 system per point; m, c carry over between levels.  Returns (flow, converged, m, c)."""
    P0, P1 = [I0], [I1]
    for _ in range(levels - 1):
        P0.append(pyr_down_scipy(P0[-1]))
        P1.append(pyr_down_scipy(P1[-1]))
    P0 = [p.astype(np.float64) for p in P0]
    P1 = [p.astype(np.float64) for p in P1]
    pts = np.asarray(pts, np.float64)
    n = len(pts)
    r = support // 2
    ky, kx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    kx, ky = kx.ravel()[None, :], ky.ravel()[None, :]
    g = np.zeros((n, 2))
    d = np.zeros((n, 2))
    m = np.zeros(n)
    c = np.zeros(n)
    conv = np.zeros(n, bool)
    for l in range(levels - 1, -1, -1):
        pl = pts / 2.0 ** l
        X, Y = pl[:, :1] + kx, pl[:, 1:] + ky
        T = _sample(P0[l], X, Y)
        GX = 0.5 * (_sample(P0[l], X + 1.0, Y) - _sample(P0[l], X - 1.0, Y))
        GY = 0.5 * (_sample(P0[l], X, Y + 1.0) - _sample(P0[l], X, Y - 1.0))
        d = np.zeros((n, 2))
        active = np.ones(n, bool)
        conv = np.zeros(n, bool)
        eps = eps_coarse if l > 0 else eps_fine
        for _ in range(iters):
            if not active.any():
                break
            J = _sample(P1[l], X + (g[:, :1] + d[:, :1]), Y + (g[:, 1:] + d[:, 1:]))
            res = J - (1.0 + m)[:, None] * T - c[:, None]
            phi = np.stack([(1.0 + m)[:, None] * GX, (1.0 + m)[:, None] * GY, -T, -np.ones_like(T)], axis=2)
            A = np.einsum("nka,nkb->nab", phi, phi)
            b = -np.einsum("nk,nka->na", res, phi)
            delta = np.linalg.solve(A, b[..., None])[..., 0]
            d[active] += delta[active, :2]
            m[active] += delta[active, 2]
            c[active] += delta[active, 3]
            done = active & (np.hypot(delta[:, 0], delta[:, 1]) < eps)
            conv |= done
            active &= ~done
        if l > 0:
            g = 2.0 * (g + d)
    return g + d, conv, m, c
