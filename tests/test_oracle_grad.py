"""Pins of the oracle's implicit gradient d(flow)/d(I0, I1) at the converged level-0 fixed point
against central finite differences of the oracle's own forward tracker (FP64).

Loss: L = sum over points CONVERGED in the forward pass of |u_k - u_gt|^2, with the points held
fixed (detection is not differentiated)."""
import numpy as np
import pytest

import oracle
from paper_1901_09971_amd import synth

LEVELS, SUPPORT = 3, 9
FD_OPTS = dict(iters=100, eps_fine=1e-12)
H_FD = 1e-3


def _loss(I0, I1, pts, gt, mask, levels=LEVELS, support=SUPPORT):
    flow, st = oracle.track(I0, I1, pts, levels, support, FD_OPTS["iters"], eps_fine=FD_OPTS["eps_fine"], threads=1)
    if not np.all(st[mask] == oracle.ST_CONVERGED):
        raise AssertionError("a point left the converged set under perturbation")
    e = flow[mask] - gt
    return float((e * e).sum())


def _setup(W, H, window, stride, crop=None):
    I0f, I1f, gt = synth.translation_f32_1242x375() if crop else synth.noise_translation_pair(W, H, seed=21, dtype="f32")
    I0 = I0f.astype(np.float64)
    I1 = I1f.astype(np.float64)
    if crop:
        x0, y0, W, H = crop
        I0 = np.ascontiguousarray(I0[y0:y0 + H, x0:x0 + W])
        I1 = np.ascontiguousarray(I1[y0:y0 + H, x0:x0 + W])
    pts, _, _ = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), window, stride)
    flow, st = oracle.track(I0, I1, pts, LEVELS, SUPPORT, FD_OPTS["iters"], eps_fine=FD_OPTS["eps_fine"])
    conv = st == oracle.ST_CONVERGED
    dflow = np.zeros_like(flow)
    dflow[conv] = 2.0 * (flow[conv] - gt)
    dI0, dI1 = oracle.track_grad(I0, I1, pts, SUPPORT, flow, st, dflow)
    return I0, I1, pts, gt, conv, flow, dI0, dI1


def _fd_full(I0, I1, pts, gt, conv, flow, image_index):
    """Central differences at every pixel; only points whose level-0 support (plus the
    interpolation and difference halo) contains the pixel are re-tracked -- coarser levels only
    choose the basin, so the other points move by far less than the tracking tolerance."""
    H, W = I0.shape
    r = SUPPORT // 2 + 3
    cen = pts if image_index == 0 else pts + flow
    fd = np.zeros((H, W))
    idx_conv = np.nonzero(conv)[0]
    for y in range(H):
        near_y = idx_conv[np.abs(cen[idx_conv, 1] - y) <= r]
        for x in range(W):
            near = near_y[np.abs(cen[near_y, 0] - x) <= r]
            if near.size == 0:
                continue
            sub_pts = pts[near]
            mask = np.ones(near.size, bool)
            imgs = [I0.copy(), I1.copy()]
            v = imgs[image_index][y, x]
            imgs[image_index][y, x] = v + H_FD
            lp = _loss(imgs[0], imgs[1], sub_pts, gt, mask)
            imgs[image_index][y, x] = v - H_FD
            lm = _loss(imgs[0], imgs[1], sub_pts, gt, mask)
            fd[y, x] = (lp - lm) / (2 * H_FD)
    return fd


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_grad_matches_fd_small():
    I0, I1, pts, gt, conv, flow, dI0, dI1 = _setup(40, 34, 9, 6)
    assert conv.sum() >= 12
    fd0 = _fd_full(I0, I1, pts, gt, conv, flow, 0)
    fd1 = _fd_full(I0, I1, pts, gt, conv, flow, 1)
    assert _rel(dI0, fd0) < 1e-5
    assert _rel(dI1, fd1) < 1e-5


@pytest.mark.slow
def test_grad_matches_fd_crop_200_points():
    # 128x64 crop at (0, 0) of the 1242x375 FP32 translation pair, window 9, stride 6: 200 points
    I0, I1, pts, gt, conv, flow, dI0, dI1 = _setup(0, 0, 9, 6, crop=(0, 0, 128, 64))
    assert len(pts) == 200
    assert conv.sum() >= 150
    fd0 = _fd_full(I0, I1, pts, gt, conv, flow, 0)
    fd1 = _fd_full(I0, I1, pts, gt, conv, flow, 1)
    assert _rel(dI0, fd0) < 1e-5
    assert _rel(dI1, fd1) < 1e-5


def test_grad_random_directions():
    I0, I1, pts, gt, conv, flow, dI0, dI1 = _setup(96, 72, 9, 7)
    rng = np.random.default_rng(3)
    for _ in range(3):
        v0 = rng.normal(size=I0.shape)
        v1 = rng.normal(size=I1.shape)
        lp = _loss(I0 + H_FD * v0, I1 + H_FD * v1, pts[conv], gt, np.ones(conv.sum(), bool))
        lm = _loss(I0 - H_FD * v0, I1 - H_FD * v1, pts[conv], gt, np.ones(conv.sum(), bool))
        fd = (lp - lm) / (2 * H_FD)
        an = float((dI0 * v0).sum() + (dI1 * v1).sum())
        assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-12) + 1e-9


def test_grad_zero_for_non_converged_and_zero_upstream():
    I0, I1, pts, gt, conv, flow, _, _ = _setup(40, 34, 9, 6)
    st = np.full(len(pts), oracle.ST_NOT_CONVERGED, np.uint8)
    dI0, dI1 = oracle.track_grad(I0, I1, pts, SUPPORT, flow, st, np.ones_like(flow))
    assert np.all(dI0 == 0) and np.all(dI1 == 0)
    st = np.zeros(len(pts), np.uint8)
    dI0, dI1 = oracle.track_grad(I0, I1, pts, SUPPORT, flow, st, np.zeros_like(flow))
    assert np.all(dI0 == 0) and np.all(dI1 == 0)


def test_grad_of_brightness_offset():
    # adding a constant to I1 inside the least-squares band: d/dc of u is -J^-1 sum psi' g, so the
    # summed gradient over all I1 pixels must equal that directional derivative
    I0, I1, pts, gt, conv, flow, dI0, dI1 = _setup(56, 48, 9, 8)
    ones = np.ones_like(I1)
    lp = _loss(I0, I1 + H_FD * ones, pts[conv], gt, np.ones(conv.sum(), bool))
    lm = _loss(I0, I1 - H_FD * ones, pts[conv], gt, np.ones(conv.sum(), bool))
    fd = (lp - lm) / (2 * H_FD)
    assert abs(dI1.sum() - fd) <= 1e-5 * abs(fd) + 1e-9


def _fallback_case(illum):
    """A pair on which many points converge in the tracker's least-squares fallback regime: I1 is
    the translated frame plus N(0, 20) noise (for the illumination model also a gain of 0.9 and an
    offset of 10), and hard thresholding at sigma = 0.5 keeps almost no residual, so the weighted
    system falls back at the converged flow."""
    I0, I1, _ = synth.noise_translation_pair(64, 48, seed=21, dtype="f32")
    I0 = I0.astype(np.float64)
    noise = np.random.default_rng(5).normal(0, 20.0, I1.shape)
    I1 = (0.9 * I1.astype(np.float64) + 10.0 if illum else I1.astype(np.float64)) + noise
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0]
    return I0, I1, pts


def _directional_checks(I0, I1, pts, illum, kw):
    """Per converged point: the gradient of lambda . u along a random image direction against the
    central difference of the forward (h = 1e-4), on the points whose perturbed forward keeps its
    status and basin (hard thresholds make the others jump)."""
    out = oracle.track(I0, I1, pts, LEVELS, SUPPORT, 100, eps_fine=1e-12, illum=illum, return_illum=illum, **kw)
    flow, st = out[0], out[1]
    lam = np.array([[0.7, -1.3]])
    h, checked, worst = 1e-4, 0, 0.0
    for i in np.nonzero(st == oracle.ST_CONVERGED)[0]:
        P = pts[i:i + 1]
        if illum:
            dI0, dI1 = oracle.track_grad_illum(I0, I1, P, SUPPORT, flow[i:i + 1], out[2][i:i + 1], st[i:i + 1], lam, **kw)
        else:
            dI0, dI1 = oracle.track_grad(I0, I1, P, SUPPORT, flow[i:i + 1], st[i:i + 1], lam, **kw)
        g = np.random.default_rng(int(i))
        v0, v1 = g.normal(size=I0.shape), g.normal(size=I1.shape)

        def fwd(a, b):
            f, s = oracle.track(a, b, P, LEVELS, SUPPORT, 100, eps_fine=1e-12, illum=illum, threads=1, **kw)
            return f[0], s[0]
        fp, sp = fwd(I0 + h * v0, I1 + h * v1)
        fm, sm = fwd(I0 - h * v0, I1 - h * v1)
        if sp != oracle.ST_CONVERGED or sm != oracle.ST_CONVERGED or np.abs(fp - fm).max() > 1e-2:
            continue
        fd = float(((fp - fm) / (2 * h) * lam[0]).sum())
        an = float((dI0 * v0).sum() + (dI1 * v1).sum())
        worst = max(worst, abs(fd - an) / max(abs(fd), 1e-9))
        checked += 1
    return checked, worst


def test_grad_least_squares_fallback_regime():
    # the gradient differentiates the equation the forward pass stopped on: at a point where the
    # weighted system falls back to least squares at the converged flow, sum r g = 0.  (A gradient
    # of the robust equation there is zero or blows up: 11 of these points, before that reading.)
    I0, I1, pts = _fallback_case(False)
    checked, worst = _directional_checks(I0, I1, pts, False, dict(sigma1=0.5, sigma2=0.5))
    assert checked >= 25 and worst < 1e-6, (checked, worst)
