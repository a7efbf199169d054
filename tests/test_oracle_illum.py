"""Pins of the oracle's illumination-model tracker (gain and offset estimated with the flow, the
RLOF(IM) configuration of Section 3 "Parameters", read as I1(p + k + u) ~ (1 + m) I0(p + k) + c)
against exact recoveries, an invariance, the fixed-point equations and an independent
least-squares implementation."""
import numpy as np
from scipy import ndimage

import oracle
from brute import lk_pyramidal_illum
from paper_1901_09971_amd import synth

INF = float("inf")


def _texture(W, H, seed, sigma=2.0):
    return synth.smoothed_noise(np.random.default_rng(seed), W, H, sigma)


def _interior(W, H, n, margin, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(margin, W - 1 - margin, n), rng.uniform(margin, H - 1 - margin, n)], 1)


def test_exact_gain_offset_and_integer_translation():
    # I1 = (1 + m0) I0 shifted by an integer t, plus c0: bilinear sampling is linear, so the model
    # has an exact zero-residual solution (d = t, m = m0, c = c0) that the iteration must reach
    W, H, t, m0, c0 = 120, 96, (3, -2), 0.25, -14.0
    I0 = _texture(W, H, 1)
    I1 = np.full_like(I0, np.nan)
    I1[max(t[1], 0):H + min(t[1], 0), max(t[0], 0):W + min(t[0], 0)] = \
        (1.0 + m0) * I0[max(-t[1], 0):H - max(t[1], 0), max(-t[0], 0):W - max(t[0], 0)] + c0
    I1 = np.where(np.isnan(I1), (1.0 + m0) * I0 + c0, I1)  # border band, outside every support
    pts = _interior(W, H, 25, 20, 2)
    for sig in ((8.0, 32.0), (INF, INF)):
        flow, st, mc = oracle.track(I0, I1, pts, 2, 9, 60, sigma1=sig[0], sigma2=sig[1], eps_fine=1e-12,
                                    min_eig=0.0, illum=True, return_illum=True)
        assert np.all(st == oracle.ST_CONVERGED)
        assert np.max(np.abs(flow - np.array(t, float))) < 1e-8
        assert np.max(np.abs(mc[:, 0] - m0)) < 1e-9 and np.max(np.abs(mc[:, 1] - c0)) < 1e-6
    # the plain tracker cannot explain the gain and offset
    flow_p, st_p = oracle.track(I0, I1, pts, 2, 9, 60, sigma1=INF, sigma2=INF, eps_fine=1e-12, min_eig=0.0)
    assert np.max(np.abs(flow_p - np.array(t, float))) > 1e-3


def test_least_squares_equals_independent_implementation():
    I0, I1, _ = synth.noise_translation_pair(128, 96, seed=3, shift=(1.6, -0.7), dtype="f32")
    I1 = 1.15 * I1.astype(np.float64) + 9.0
    pts = _interior(128, 96, 40, 14, 4)
    flow, st, mc = oracle.track(I0.astype(np.float64), I1, pts, 3, 9, 30, sigma1=INF, sigma2=INF, min_eig=0.0,
                                illum=True, return_illum=True)
    bflow, bconv, bm, bc = lk_pyramidal_illum(I0.astype(np.float64), I1, pts, 3, 9, 30, 1e-2, 1e-4)
    assert np.array_equal(st == oracle.ST_CONVERGED, bconv)
    assert np.max(np.abs(flow - bflow)) < 1e-9
    assert np.max(np.abs(mc[:, 0] - bm)) < 1e-9 and np.max(np.abs(mc[:, 1] - bc)) < 1e-7


def test_least_squares_invariant_to_gain_and_offset_of_I1():
    # with residual derivatives ((1 + m) g, -T, -1), Gauss-Newton is invariant under
    # I1 -> a I1 + b (the parameters map to (a (1 + m) - 1, a c + b)); the robust weights are not
    I0, I1, _ = synth.noise_translation_pair(128, 96, seed=5, shift=(-2.3, 1.1), dtype="f32")
    I0, I1 = I0.astype(np.float64), I1.astype(np.float64)
    pts = _interior(128, 96, 40, 14, 6)
    # converged to round-off, so that no stopping decision sits on the eps boundary
    kw = dict(sigma1=INF, sigma2=INF, min_eig=0.0, eps_coarse=1e-12, eps_fine=1e-12, illum=True, return_illum=True)
    f1, s1, mc1 = oracle.track(I0, I1, pts, 3, 9, 80, **kw)
    a, b = 1.3, -17.0
    f2, s2, mc2 = oracle.track(I0, a * I1 + b, pts, 3, 9, 80, **kw)
    assert np.array_equal(s1, s2)
    assert np.max(np.abs(f1 - f2)) < 1e-8
    assert np.max(np.abs(mc2[:, 0] - (a * (1.0 + mc1[:, 0]) - 1.0))) < 1e-8
    assert np.max(np.abs(mc2[:, 1] - (a * mc1[:, 1] + b))) < 1e-6


def test_robust_fixed_point():
    # at a converged point sum_k psi(r_k) phi_k = 0 in all four components, evaluated here from
    # scratch with the returned flow, m and c; the middle band of psi is active
    I0, I1, _, _ = synth.layered_pair(160, 120, seed=7, max_disp=12.0, dtype="f32")
    I0, I1 = I0.astype(np.float64), 0.9 * I1.astype(np.float64) + 12.0
    pts = _interior(160, 120, 60, 15, 8)
    s1_, s2_ = 8.0, 32.0
    flow, st, mc = oracle.track(I0, I1, pts, 1, 11, 200, eps_fine=1e-13, min_eig=0.0, illum=True,
                                return_illum=True)
    conv = np.where(st == oracle.ST_CONVERGED)[0]
    assert len(conv) > 30
    r = 5
    ky, kx = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    mid = 0
    for i in conv:
        X, Y = pts[i, 0] + kx, pts[i, 1] + ky
        smp = lambda img, x, y: ndimage.map_coordinates(img, [y.ravel(), x.ravel()], order=1, mode="nearest")
        T = smp(I0, X, Y)
        gx = 0.5 * (smp(I0, X + 1, Y) - smp(I0, X - 1, Y))
        gy = 0.5 * (smp(I0, X, Y + 1) - smp(I0, X, Y - 1))
        J = smp(I1, X + flow[i, 0], Y + flow[i, 1])
        m, c = mc[i]
        res = J - (1.0 + m) * T - c
        a = np.abs(res)
        psi = np.where(a <= s1_, res, np.where(a >= s2_, 0.0, np.sign(res) * s1_ * (s2_ - a) / (s2_ - s1_)))
        mid += int(np.sum((a > s1_) & (a < s2_)))
        F = np.array([np.sum(psi * (1 + m) * gx), np.sum(psi * (1 + m) * gy), -np.sum(psi * T), -np.sum(psi)])
        scale = np.sum(np.abs(psi)) * (np.abs(gx).max() + np.abs(gy).max() + np.abs(T).max() + 1.0)
        assert np.max(np.abs(F)) <= 1e-8 * scale
    assert mid > 0


def test_no_illumination_change_stays_close_to_plain():
    I0, I1, gt = synth.noise_translation_pair(160, 120, seed=9, shift=(2.2, -1.4))
    pts = _interior(160, 120, 50, 15, 10)
    fp, sp = oracle.track(I0, I1, pts, 3, 9, 20)
    fi, si, mc = oracle.track(I0, I1, pts, 3, 9, 20, illum=True, return_illum=True)
    both = (sp == oracle.ST_CONVERGED) & (si == oracle.ST_CONVERGED)
    assert both.mean() > 0.8
    ep = np.median(np.linalg.norm(fp[both] - gt, axis=1))
    ei = np.median(np.linalg.norm(fi[both] - gt, axis=1))
    assert ei < 0.1 and ei < 2.0 * ep + 0.02  # two more unknowns, about the same accuracy
    # gain and offset trade off against each other; their effect at the support's mean intensity
    # stays near zero
    ky, kx = np.mgrid[-4:5, -4:5]
    Tm = np.array([ndimage.map_coordinates(I0.astype(np.float64), [p[1] + ky.ravel(), p[0] + kx.ravel()],
                                           order=1).mean() for p in pts])
    assert np.max(np.abs(mc[both, 0] * Tm[both] + mc[both, 1])) < 1.5


def test_large_offset_takes_the_least_squares_step_first():
    # every residual of the first step lies beyond sigma2 (an offset of 60 on a low-contrast
    # texture), so all robust weights vanish and the weighted matrix is singular: only the
    # least-squares fallback can take the first step, after which the offset is absorbed by c
    W, H, t = 100, 80, (2, 1)
    I0 = 90.0 + _texture(W, H, 11) * (20.0 / 255.0)
    I1 = np.empty_like(I0)
    I1[t[1]:, t[0]:] = I0[:H - t[1], :W - t[0]] + 60.0
    I1[:t[1], :] = I0[:t[1], :] + 60.0
    I1[:, :t[0]] = I0[:, :t[0]] + 60.0
    pts = _interior(W, H, 20, 18, 12)
    flow, st, mc = oracle.track(I0, I1, pts, 1, 9, 40, eps_fine=1e-10, min_eig=0.0, illum=True, return_illum=True)
    assert np.all(st == oracle.ST_CONVERGED)
    assert np.max(np.abs(flow - np.array(t, float))) < 1e-6
    assert np.max(np.abs(mc[:, 0] * 100.0 + mc[:, 1] - 60.0)) < 1e-3


def test_contrast_inversion_is_not_a_match():
    # I1 = 255 - I0 shifted: the model fits it exactly with gain -1, which is a contrast inversion,
    # not an illumination change; such points end NOT_CONVERGED (gain outside [1/2, 2])
    W, H, t = 100, 80, (2, -1)
    I0 = _texture(W, H, 13)
    I1 = 255.0 - I0
    I1[max(t[1], 0):H + min(t[1], 0), max(t[0], 0):W + min(t[0], 0)] = \
        255.0 - I0[max(-t[1], 0):H - max(t[1], 0), max(-t[0], 0):W - max(t[0], 0)]
    pts = _interior(W, H, 15, 18, 14)
    flow, st, mc = oracle.track(I0, I1, pts, 1, 9, 60, sigma1=INF, sigma2=INF, eps_fine=1e-10, min_eig=0.0,
                                illum=True, return_illum=True)
    exact = np.abs(1.0 + mc[:, 0] + 1.0) < 1e-6  # points that reached the exact fit, gain -1
    assert exact.sum() >= 5 and np.max(np.abs(flow[exact] - np.array(t, float))) < 1e-6
    assert np.all(st[exact] == oracle.ST_NOT_CONVERGED)
    # a gain of 1.9 stays a match
    I2 = 1.9 * I0
    flow, st = oracle.track(I0, I2, pts, 1, 9, 60, sigma1=INF, sigma2=INF, eps_fine=1e-10, min_eig=0.0, illum=True)
    assert np.all(st == oracle.ST_CONVERGED) and np.max(np.abs(flow)) < 1e-8


def test_implicit_gradient_matches_finite_differences():
    # L = sum over converged points of lam . u for the illumination-model tracker (one level,
    # converged to round-off), against central differences pixel by pixel on a small crop of both
    # frames; the gain and offset differ from (0, 0) and the robust middle band is active
    I0, I1, _ = synth.noise_translation_pair(44, 40, seed=17, shift=(0.7, -0.4), dtype="f32")
    I0 = I0.astype(np.float64)
    I1 = 1.1 * I1.astype(np.float64) - 9.0 + 6.0 * np.sin(np.arange(44) / 5.0)[None, :]
    rng = np.random.default_rng(18)
    pts = np.stack([rng.uniform(12, 31, 6), rng.uniform(12, 27, 6)], 1)
    kw = dict(eps_fine=1e-13, min_eig=0.0, illum=True)
    flow, st, mc = oracle.track(I0, I1, pts, 1, 9, 400, return_illum=True, **kw)
    assert np.all(st == oracle.ST_CONVERGED)
    lam = rng.normal(size=flow.shape)
    g0, g1 = oracle.track_grad_illum(I0, I1, pts, 9, flow, mc, st, lam)
    h = 1e-5
    for img, g in ((I0, g0), (I1, g1)):
        ys, xs = np.nonzero(np.abs(g) > 1e-9 * np.abs(g).max())
        pick = rng.choice(len(ys), 60, replace=False)
        for y, x in zip(ys[pick], xs[pick]):
            vals = []
            for sgn in (1.0, -1.0):
                a = img.copy()
                a[y, x] += sgn * h
                f, s = oracle.track(a if img is I0 else I0, a if img is I1 else I1, pts, 1, 9, 400, **kw)
                assert np.array_equal(s, st)
                vals.append(np.sum(lam * f))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(g[y, x] - fd) <= 1e-5 * np.abs(g).max(), (y, x, g[y, x], fd)


def test_point_gradient_matches_finite_differences():
    # dL/dp of the illumination-model tracker (the template moves with the point) against central
    # differences of the forward in the point positions; gain and offset away from (0, 0), the
    # robust middle band active
    I0, I1, _ = synth.noise_translation_pair(72, 60, seed=5, shift=(1.3, -0.8), dtype="f32")
    I0 = I0.astype(np.float64)
    I1 = 0.9 * I1.astype(np.float64) + 11.0 + 3.0 * np.sin(np.arange(72) / 7.0)[None, :]
    rng = np.random.default_rng(16)
    pts = np.stack([rng.uniform(15, 56, 10), rng.uniform(15, 44, 10)], 1)
    kw = dict(eps_fine=1e-13, min_eig=0.0, illum=True)
    flow, st, mc = oracle.track(I0, I1, pts, 1, 9, 400, return_illum=True, **kw)
    assert np.mean(st == 0) > 0.8
    lam = rng.normal(size=flow.shape) * (st == 0)[:, None]
    _, _, dp = oracle.track_grad_illum(I0, I1, pts, 9, flow, mc, st, lam, return_dpoints=True)
    h = 1e-5
    for i in np.where(st == 0)[0]:
        for c in range(2):
            a = pts.copy()
            a[i, c] += h
            fa, _ = oracle.track(I0, I1, a[i:i + 1], 1, 9, 400, **kw)
            b = pts.copy()
            b[i, c] -= h
            fb, _ = oracle.track(I0, I1, b[i:i + 1], 1, 9, 400, **kw)
            fd = float(np.sum(lam[i] * (fa[0] - fb[0])) / (2 * h))
            assert abs(dp[i, c] - fd) <= 1e-5 * (abs(fd) + np.abs(lam[i]).sum()), (i, c, dp[i, c], fd)
    assert np.all(dp[st != 0] == 0.0)


def test_coarse_level_with_a_runaway_gain_ends_the_point():
    # the contrast-inverted pair on two levels: the coarse level already fits gain -1, outside
    # [1/4, 4], so the point ends there (NOT_CONVERGED, NaN flow) instead of carrying an inverted
    # model to the finer level
    W, H, t = 100, 80, (2, -1)
    I0 = _texture(W, H, 13)
    I1 = 255.0 - I0
    I1[max(t[1], 0):H + min(t[1], 0), max(t[0], 0):W + min(t[0], 0)] = \
        255.0 - I0[max(-t[1], 0):H - max(t[1], 0), max(-t[0], 0):W - max(t[0], 0)]
    pts = _interior(W, H, 15, 18, 14)
    kw = dict(sigma1=INF, sigma2=INF, eps_fine=1e-10, min_eig=0.0, illum=True)
    flow, st, its, mc = oracle.track(I0, I1, pts, 2, 9, 60, return_iters=True, return_illum=True, **kw)
    ended = np.isnan(flow).all(1)
    assert ended.sum() >= 10 and np.all(st[ended] == oracle.ST_NOT_CONVERGED)
    assert np.all(its[ended, 1] == 0) and np.all(1.0 + mc[ended, 0] < 0.25)  # stopped before level 0
    # a gain of 1.9 stays a match through both levels
    flow, st = oracle.track(I0, 1.9 * I0, pts, 2, 9, 60, **kw)
    assert np.all(st == oracle.ST_CONVERGED) and np.max(np.abs(flow)) < 1e-8


def test_cross_support_of_fewer_than_four_pixels_is_flat_for_the_illumination_model():
    # a 3 x 4 block of mutually similar values on a far brighter frame: the cross region at the
    # block's centre is the block, and the gradient-stencil erosion keeps two pixels -- enough for
    # the 2 x 2 system of the plain tracker, too few for the four unknowns of the illumination model
    W = H = 40
    I0 = np.full((H, W), 200.0)
    I0[19:22, 19:23] = np.array([[100.0, 108.0, 95.0, 104.0], [112.0, 99.0, 110.0, 93.0], [97.0, 115.0, 102.0, 109.0]])
    I1 = np.roll(I0, (1, 1), axis=(0, 1))
    p = np.array([[20.3, 20.2]])
    ys, xs = np.arange(20 - 11, 20 + 12), np.arange(20 - 11, 20 + 12)
    m = oracle.cross_mask(I0[np.ix_(np.clip(ys, 0, H - 1), np.clip(xs, 0, W - 1))])
    assert m.sum() == 2 and m[10, 10] and m[10, 11]
    kw = dict(cross=True, min_eig=0.0)
    f, st = oracle.track(I0, I1, p, 1, 21, 20, **kw)
    assert st[0] != oracle.ST_ILL_CONDITIONED
    f, st = oracle.track(I0, I1, p, 1, 21, 20, illum=True, **kw)
    assert st[0] == oracle.ST_ILL_CONDITIONED


def test_grad_illum_least_squares_fallback_regime():
    # as for the plain tracker: in the least-squares fallback regime of the 4 x 4 system at the
    # converged (u, m, c) the gradient differentiates the least-squares equations (49 of these 54
    # points had a wrong gradient of the robust equations)
    from test_oracle_grad import _directional_checks, _fallback_case
    I0, I1, pts = _fallback_case(True)
    checked, worst = _directional_checks(I0, I1, pts, True, dict(sigma1=0.5, sigma2=0.5))
    assert checked >= 40 and worst < 1e-6, (checked, worst)
