"""Seeded synthetic frame pairs with known ground-truth motion.

This module only *generates inputs*: it contains none of the method's arithmetic (no key-point
detection, no pyramid, no tracking).  Smoothing and resampling are done with scipy.ndimage so
that neither the HIP path nor the CPU oracle shares code with the generator.

The paper evaluates on KITTI 2012/2015 road scenes (about 1240x376, large horizontal motion near
the image edges, occlusions at object borders; Section 3).  Those datasets are not available
here, so these generators stand in for them with procedurally textured frames of the same
shapes and motion character.  No dataset item is reproduced.

Recipes (all randomness from ``numpy.random.default_rng(seed)``):

* ``noise_translation_pair``: uniform noise U[0, 256), Gaussian smoothing (sigma 2, truncate 4,
  reflect), min-max stretch to [0, 255]; I1(x, y) = bilinear(I0, x - tx, y - ty) (clamped) plus
  N(0, 1) noise.  Ground-truth flow is (tx, ty) everywhere.  uint8 (rounded, clipped) or float32.
* ``layered_pair``: a "driving-shaped" scene of six layers painted back to front -- far band,
  road, left and right roadside wedges and two vehicle boxes -- each with its own texture
  (smoothed noise of a random scale plus a linear ramp) and its own affine motion.  Far band and
  road-side layers expand about a focus of expansion at (W/2, 0.42 H); the expansion is chosen so
  that the horizontal displacement reaches ``max_disp`` pixels at the left/right image edges.
  I1 is rendered by inverse-affine sampling of each layer (front layer wins), so occlusions fall
  at layer borders; N(0, 1) noise is added to I1.  Ground truth is the affine flow of the layer
  that owns each I0 pixel, plus an occlusion flag.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import ndimage


def _stretch(a: np.ndarray, lo: float = 0.0, hi: float = 255.0) -> np.ndarray:
    mn, mx = float(a.min()), float(a.max())
    if mx <= mn:
        return np.full_like(a, (lo + hi) / 2.0)
    return lo + (a - mn) * ((hi - lo) / (mx - mn))


def _to_u8(a: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(a), 0, 255).astype(np.uint8)


def smoothed_noise(rng: np.random.Generator, W: int, H: int, sigma: float) -> np.ndarray:
    noise = rng.uniform(0.0, 256.0, size=(H, W))
    sm = ndimage.gaussian_filter(noise, sigma=sigma, mode="reflect", truncate=4.0)
    return _stretch(sm)


def noise_translation_pair(W: int, H: int, seed: int = 0, shift=(2.3, -1.7), sigma: float = 2.0,
                           dtype: str = "u8"):
    """Returns (I0, I1, gt_flow (2,)) -- see module docstring."""
    rng = np.random.default_rng(seed)
    I0f = smoothed_noise(rng, W, H, sigma)
    if dtype == "u8":
        I0f = np.rint(np.clip(I0f, 0, 255))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    tx, ty = shift
    I1f = ndimage.map_coordinates(I0f, [yy - ty, xx - tx], order=1, mode="nearest")
    I1f = I1f + rng.normal(0.0, 1.0, size=(H, W))
    if dtype == "u8":
        return I0f.astype(np.uint8), _to_u8(I1f), np.array(shift, np.float64)
    return I0f.astype(np.float32), I1f.astype(np.float32), np.array(shift, np.float64)


@dataclass
class Layer:
    kind: str
    region: object          # callable (x, y) -> bool mask, in I0 coordinates
    A: np.ndarray           # 2x2 linear part: q = A @ (p - c) + c + t
    c: np.ndarray           # centre of the linear part
    t: np.ndarray           # translation
    tex: np.ndarray         # texture canvas, I0 coordinates, float64 [H][W]

    def forward(self, x, y):
        dx, dy = x - self.c[0], y - self.c[1]
        qx = self.A[0, 0] * dx + self.A[0, 1] * dy + self.c[0] + self.t[0]
        qy = self.A[1, 0] * dx + self.A[1, 1] * dy + self.c[1] + self.t[1]
        return qx, qy

    def inverse(self, qx, qy):
        Ai = np.linalg.inv(self.A)
        dx, dy = qx - self.c[0] - self.t[0], qy - self.c[1] - self.t[1]
        return Ai[0, 0] * dx + Ai[0, 1] * dy + self.c[0], Ai[1, 0] * dx + Ai[1, 1] * dy + self.c[1]


def _layers(rng: np.random.Generator, W: int, H: int, max_disp: float):
    horizon = 0.42 * H
    foe = np.array([W / 2.0, horizon])
    s_road = 1.0 + max_disp / (W / 2.0)
    k = W / 1242.0  # scale the vehicle motion with the frame width

    def tex():
        sigma = float(rng.choice([1.0, 1.5, 2.0, 3.0, 4.0]))
        base = smoothed_noise(rng, W, H, sigma)
        theta = rng.uniform(0, 2 * np.pi)
        amp = rng.uniform(20.0, 80.0)
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
        ramp = amp * (np.cos(theta) * xx / W + np.sin(theta) * yy / H)
        lo = rng.uniform(0.0, 40.0)
        hi = rng.uniform(215.0, 255.0)
        return _stretch(base + ramp, lo, hi)

    I2 = np.eye(2)
    L = []
    L.append(Layer("far", lambda x, y: np.ones_like(x, dtype=bool), 1.01 * I2, foe, np.zeros(2), tex()))
    L.append(Layer("road", lambda x, y: y >= horizon, s_road * I2, foe, np.zeros(2), tex()))
    wedge_w = 0.30 * W

    def left(x, y):
        return (y >= horizon) & (x < wedge_w * (y - horizon) / (H - horizon))

    def right(x, y):
        return (y >= horizon) & (x > W - 1 - wedge_w * (y - horizon) / (H - horizon))

    L.append(Layer("left", left, s_road * I2, foe, np.zeros(2), tex()))
    L.append(Layer("right", right, s_road * I2, foe, np.zeros(2), tex()))
    # two vehicles: boxes with their own translation and scale about the box centre
    for (x0, x1, y0, y1, t, s) in ((0.14, 0.33, 0.45, 0.80, (-22.0 * k, 2.5 * k), 1.06),
                                   (0.58, 0.72, 0.40, 0.62, (13.0 * k, -1.2 * k), 0.97)):
        bx0, bx1, by0, by1 = x0 * W, x1 * W, y0 * H, y1 * H
        c = np.array([(bx0 + bx1) / 2.0, (by0 + by1) / 2.0])
        L.append(Layer("vehicle", (lambda a0, a1, b0, b1: (lambda x, y: (x >= a0) & (x <= a1) & (y >= b0) & (y <= b1)))(
            bx0, bx1, by0, by1), s * I2, c, np.array(t), tex()))
    return L


def layered_pair(W: int, H: int, seed: int = 0, max_disp: float = 150.0, dtype: str = "u8"):
    """Returns (I0, I1, gt_flow[H][W][2] float64, occluded[H][W] bool) -- see module docstring."""
    rng = np.random.default_rng(seed)
    layers = _layers(rng, W, H, max_disp)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    # I0: front-most layer whose region contains the pixel
    owner0 = np.zeros((H, W), np.int32)
    for i, ly in enumerate(layers):
        owner0[ly.region(xx, yy)] = i
    I0 = np.zeros((H, W), np.float64)
    for i, ly in enumerate(layers):
        m = owner0 == i
        I0[m] = ly.tex[m]

    # I1: front-most layer whose back-projected position lies in its own region
    I1 = np.zeros((H, W), np.float64)
    owner1 = np.zeros((H, W), np.int32)
    for i, ly in enumerate(layers):
        sx, sy = ly.inverse(xx, yy)
        m = ly.region(sx, sy)
        vals = ndimage.map_coordinates(ly.tex, [sy, sx], order=1, mode="nearest")
        I1[m] = vals[m]
        owner1[m] = i

    # ground truth: affine flow of the I0 owner; occluded if a front layer covers the target
    gt = np.zeros((H, W, 2), np.float64)
    for i, ly in enumerate(layers):
        m = owner0 == i
        qx, qy = ly.forward(xx, yy)
        gt[..., 0][m] = (qx - xx)[m]
        gt[..., 1][m] = (qy - yy)[m]
    qx, qy = xx + gt[..., 0], yy + gt[..., 1]
    inside = (qx >= 0) & (qy >= 0) & (qx <= W - 1) & (qy <= H - 1)
    qi = np.clip(np.rint(qx), 0, W - 1).astype(np.int64)
    qj = np.clip(np.rint(qy), 0, H - 1).astype(np.int64)
    occluded = ~inside | (owner1[qj, qi] > owner0)

    I1 = I1 + rng.normal(0.0, 1.0, size=(H, W))
    if dtype == "u8":
        return _to_u8(I0), _to_u8(I1), gt, occluded
    return I0.astype(np.float32), I1.astype(np.float32), gt, occluded


# --------------------------------------------------------------------------------------------
# The five workloads.  Tracker settings per workload; window 9 everywhere.
# --------------------------------------------------------------------------------------------

WORKLOADS = {
    "translation_256x128": dict(W=256, H=128, window=9, stride=8, levels=3, support=9, iters=10),
    "driving_1242x375": dict(W=1242, H=375, window=9, stride=5, levels=5, support=21, iters=20),
    "batch64_mixed": dict(window=9, levels=5, support=21, iters=20),
    "translation_f32_1242x375": dict(W=1242, H=375, window=9, stride=8, levels=3, support=9, iters=10),
    "density_2048x1024x4": dict(W=2048, H=1024, window=9, stride=2, levels=6, support=21, iters=20),
}


def translation_256x128(seed: int = 0):
    return noise_translation_pair(256, 128, seed=seed)


def driving_1242x375(seed: int = 0):
    return layered_pair(1242, 375, seed=seed, max_disp=150.0)


def batch64_mixed(workers: int = 8):
    """64 pairs of four sizes (16 each), pair i uses seed i, stride per pair drawn from
    {3, 5, 8} with rng(0).  Returns a list of dicts (I0, I1, gt, occ, stride).  Pairs are
    generated on a thread pool (each pair has its own generator, so the result does not depend
    on the scheduling)."""
    from concurrent.futures import ThreadPoolExecutor
    sizes = [(1242, 375), (1224, 370), (640, 480), (320, 240)]
    strides = np.random.default_rng(0).choice([3, 5, 8], size=64)

    def one(i):
        W, H = sizes[i % 4]
        I0, I1, gt, occ = layered_pair(W, H, seed=i, max_disp=150.0 * W / 1242.0)
        return dict(I0=I0, I1=I1, gt=gt, occ=occ, stride=int(strides[i]), W=W, H=H)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, range(64)))


def translation_f32_1242x375(seed: int = 0):
    return noise_translation_pair(1242, 375, seed=seed, dtype="f32")


def density_2048x1024(seed: int):
    return layered_pair(2048, 1024, seed=seed, max_disp=250.0)
