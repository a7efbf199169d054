"""Pins of the gradient through detection (the centroid ratios of Section 2 Eq. 1-2 are smooth in
the pixel values away from ties) and of the gradient of the tracked flow w.r.t. the point
positions: both against central finite differences of the oracle's own forward functions, and the
real-valued detector against the integer one."""
import numpy as np

import oracle
from paper_1901_09971_amd import synth


def test_real_detector_equals_integer_detector_on_integer_images():
    I0, _, _ = synth.translation_256x128()
    p8, s8, _ = oracle.detect(I0, 9, 8)
    pr, sr = oracle.detect_real(I0.astype(np.float64), 9, 8)
    assert np.array_equal(s8, sr)
    assert np.max(np.abs(p8 - pr)) < 1e-12


def test_detection_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    img = rng.uniform(0.0, 255.0, size=(30, 34))
    w, d = 9, 5
    pts, sel = oracle.detect_real(img, w, d)
    assert sel.min() == 0 and sel.max() == 1  # both centroids are exercised
    lam = rng.normal(size=pts.shape)
    g = oracle.detect_grad(img, w, d, sel, lam)
    h = 1e-6
    fd = np.zeros_like(img)
    for y in range(img.shape[0]):
        for x in range(img.shape[1]):
            a = img.copy()
            a[y, x] += h
            pa, sa = oracle.detect_real(a, w, d)
            b = img.copy()
            b[y, x] -= h
            pb, sb = oracle.detect_real(b, w, d)
            assert np.array_equal(sa, sel) and np.array_equal(sb, sel)
            fd[y, x] = np.sum(lam * (pa - pb)) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))
    # the window maximum enters the negative centroid: its pixels carry the extra term
    assert np.count_nonzero(g) == np.count_nonzero(fd)


def _pair(W, H, seed, shift):
    I0, I1, _ = synth.noise_translation_pair(W, H, seed=seed, shift=shift, dtype="f32")
    return I0.astype(np.float64), I1.astype(np.float64)


def test_point_gradient_of_the_flow_matches_finite_differences():
    I0, I1 = _pair(72, 60, 5, (1.3, -0.8))
    I1 = I1 + 3.0 * np.sin(np.arange(72) / 7.0)[None, :]  # residuals in the robust middle band too
    rng = np.random.default_rng(6)
    pts = np.stack([rng.uniform(15, 56, 12), rng.uniform(15, 44, 12)], 1)
    kw = dict(eps_fine=1e-13, min_eig=0.0)
    flow, st = oracle.track(I0, I1, pts, 1, 9, 300, **kw)
    assert np.mean(st == 0) > 0.8
    lam = rng.normal(size=flow.shape) * (st == 0)[:, None]
    _, _, dp = oracle.track_grad(I0, I1, pts, 9, flow, st, lam, return_dpoints=True)
    h = 1e-5
    for i in np.where(st == 0)[0]:
        for c in range(2):
            a = pts.copy()
            a[i, c] += h
            fa, sa = oracle.track(I0, I1, a[i:i + 1], 1, 9, 300, **kw)
            b = pts.copy()
            b[i, c] -= h
            fb, sb = oracle.track(I0, I1, b[i:i + 1], 1, 9, 300, **kw)
            fd = float(np.sum(lam[i] * (fa[0] - fb[0])) / (2 * h))
            assert abs(dp[i, c] - fd) <= 1e-5 * (abs(fd) + np.abs(lam[i]).sum()), (i, c, dp[i, c], fd)
    assert np.all(dp[st != 0] == 0.0)


def test_detect_and_track_gradient_end_to_end():
    # L(I0) = sum over converged points of lam . u, with the points detected on I0 (real-valued):
    # dL/dI0 = (points held) + (through the points) = track_grad dI0 + detect_grad(dL/dp)
    I0, I1 = _pair(60, 48, 7, (0.9, 0.6))
    w, d = 9, 6
    kw = dict(eps_fine=1e-13, min_eig=0.0)
    pts, sel = oracle.detect_real(I0, w, d)
    flow, st = oracle.track(I0, I1, pts, 1, 9, 300, **kw)
    rng = np.random.default_rng(8)
    lam = rng.normal(size=flow.shape) * (st == 0)[:, None]
    dI0, _, dp = oracle.track_grad(I0, I1, pts, 9, flow, st, lam, return_dpoints=True)
    total = dI0 + oracle.detect_grad(I0, w, d, sel, dp)
    h = 1e-5
    ys, xs = np.nonzero(np.abs(total) > 0)
    pick = rng.choice(len(ys), 40, replace=False)
    for y, x in zip(ys[pick], xs[pick]):
        vals = []
        for sgn in (1.0, -1.0):
            a = I0.copy()
            a[y, x] += sgn * h
            pa, sa = oracle.detect_real(a, w, d)
            fa, ta = oracle.track(a, I1, pa, 1, 9, 300, **kw)
            assert np.array_equal(sa, sel) and np.array_equal(ta, st)
            vals.append(np.sum(lam * fa))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(total[y, x] - fd) <= 1e-4 * np.max(np.abs(total)), (y, x, total[y, x], fd)
