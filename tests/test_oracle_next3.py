"""Pins of the oracle's adaptive cross-based supports and global-motion prior (the rest of the
tracker configuration RLOF(IM-GM), Section 3 "Parameters"): the mask against an independent
brute-force statement of the cross construction, the robust global fit against exact and
degenerate cases, and tracking cases whose answer is exact."""
import numpy as np
import pytest

import oracle
from paper_1901_09971_amd import synth

TAU = oracle.CROSS_TAU


def _mask_brute(Tx, tau):
    """On the (s+2)^2 extension: a pixel is in the region iff every centre-column pixel after the
    centre up to its row is within tau of the centre, and every pixel of its row after the centre
    column up to it is within tau of that row's centre-column pixel (anchors are in).  A support
    pixel is kept iff it and its four neighbours are in the region."""
    e = Tx.shape[0]
    c = e // 2
    R = np.zeros((e, e), bool)
    for ky in range(-c, c + 1):
        step = 1 if ky >= 0 else -1
        if not all(abs(Tx[c + j, c] - Tx[c, c]) <= tau for j in range(step, ky + step, step)):
            continue
        for kx in range(-c, c + 1):
            sx = 1 if kx >= 0 else -1
            if all(abs(Tx[c + ky, c + i] - Tx[c + ky, c]) <= tau for i in range(sx, kx + sx, sx)):
                R[c + ky, c + kx] = True
    inner = R[1:-1, 1:-1] & R[:-2, 1:-1] & R[2:, 1:-1] & R[1:-1, :-2] & R[1:-1, 2:]
    return inner.astype(np.uint8)


def test_cross_mask_equals_brute_force_on_random_templates():
    rng = np.random.default_rng(7)
    for t in range(300):
        s = int(rng.choice([1, 3, 5, 7, 9, 11, 15, 21]))
        e = s + 2
        kind = t % 4
        if kind == 0:
            Tx = rng.uniform(0, 255, (e, e))
        elif kind == 1:
            Tx = synth.smoothed_noise(rng, e, e, float(rng.uniform(0.5, 3)))
        elif kind == 2:  # integer levels, many exact ties with tau
            Tx = rng.integers(0, 4, (e, e)).astype(np.float64) * TAU / 2
        else:  # smooth with a pasted block and a non-finite pixel
            Tx = synth.smoothed_noise(rng, e, e, 2.0) * 0.2 + 100
            y, x = rng.integers(0, e, 2)
            Tx[y:y + 3, x:x + 4] = 200
            Tx[rng.integers(0, e), rng.integers(0, e)] = np.nan
        tau = float(rng.choice([TAU, 5.0, 60.0]))
        got = oracle.cross_mask(Tx, tau)
        assert np.array_equal(got, _mask_brute(Tx, tau)), (t, s, kind)


def test_cross_mask_hand_cases():
    s, r = 9, 4
    e = s + 2
    assert oracle.cross_mask(np.full((e, e), 77.0)).all()
    # a vertical step of 30 > tau: the columns beyond it and the column before it (whose gradient
    # would straddle the step) drop out
    T = np.full((e, e), 100.0)
    T[:, r + 1 + 3:] = 130.0
    m = oracle.cross_mask(T)
    assert m[:, :r + 2].all() and not m[:, r + 2:].any()
    # a block at the top right drops out with the rest of its rows' arms beyond it, and with the
    # pixels whose gradient stencil would reach into what dropped out
    T = np.full((e, e), 100.0)
    T[0:3, 6:8] = 200.0
    m = oracle.cross_mask(T)
    assert m[0:2, :4].all() and not m[0:2, 4:].any()
    assert m[2, :5].all() and not m[2, 5:].any() and m[3:, :].all()
    # a barrier row above the centre cuts off everything above it, even pixels equal to the centre
    T = np.full((e, e), 100.0)
    T[r + 1 - 2, :] = 180.0
    m = oracle.cross_mask(T)
    assert not m[:r, :].any() and m[r:, :].all()
    # exactly tau apart is inside
    T = np.full((e, e), 100.0)
    T[:, 0] = 100.0 + TAU
    assert oracle.cross_mask(T).all()
    # a non-finite centre keeps only the centre's own row and column arms out: nothing survives
    T = np.full((e, e), 100.0)
    T[r + 1, r + 1] = np.nan
    assert not oracle.cross_mask(T).any()


def test_gm_fit_recovers_an_exact_affine_motion_despite_outliers():
    rng = np.random.default_rng(3)
    n = 2000
    P = np.stack([rng.uniform(0, 1241, n), rng.uniform(0, 374, n)], 1)
    c = (620.5, 187.0)
    A = np.array([[0.12, -0.03, 4.5], [0.02, 0.2, -1.25]])
    V = np.einsum("ij,nj->ni", A, np.column_stack([P[:, 0] - c[0], P[:, 1] - c[1], np.ones(n)]))
    out = rng.random(n) < 0.2
    V[out] += rng.uniform(200, 400, (out.sum(), 2)) * rng.choice([-1, 1], (out.sum(), 2))
    use = np.ones(n, np.uint8)
    use[rng.random(n) < 0.1] = 0
    V[use == 0] = 1e6  # not a sample: never read into the fit
    Ag, kind = oracle.gm_fit(P, V, use, c, scale=16.0)
    assert kind == 2
    assert np.abs(Ag - A).max() < 1e-9


def test_gm_fit_plain_least_squares_without_outliers_and_degenerate_cases():
    rng = np.random.default_rng(5)
    n = 300
    P = np.stack([rng.uniform(0, 300, n), rng.uniform(0, 200, n)], 1)
    V = rng.normal(0, 0.5, (n, 2)) + [3.0, -2.0]
    c = (150.0, 100.0)
    # zero reweightings: ordinary least squares, equal to numpy's
    Ag, kind = oracle.gm_fit(P, V, np.ones(n, np.uint8), c, scale=1000.0, iters=0)
    X = np.column_stack([P[:, 0] - c[0], P[:, 1] - c[1], np.ones(n)])
    ref = np.linalg.lstsq(X, V, rcond=None)[0].T
    assert kind == 2 and np.abs(Ag - ref).max() < 1e-10
    # one row of points: positions degenerate -> the mean motion (before any reweighting), and
    # after reweighting the Tukey-weighted mean
    Pr = np.stack([np.linspace(0, 300, 50), np.full(50, 40.0)], 1)
    Ag, kind = oracle.gm_fit(Pr, V[:50], np.ones(50, np.uint8), c, scale=16.0, iters=0)
    assert kind == 1
    assert np.abs(Ag[:, :2]).max() == 0 and np.abs(Ag[:, 2] - V[:50].mean(0)).max() < 1e-12
    Ag, kind = oracle.gm_fit(Pr, V[:50], np.ones(50, np.uint8), c, scale=16.0, iters=1)
    e = np.linalg.norm(V[:50] - V[:50].mean(0), axis=1) / (4.685 * 16.0)
    w = (1 - e ** 2) ** 2
    assert kind == 1 and np.abs(Ag[:, 2] - (w[:, None] * V[:50]).sum(0) / w.sum()).max() < 1e-12
    # two samples -> translation; no sample -> no model
    Ag, kind = oracle.gm_fit(P[:2], V[:2], np.ones(2, np.uint8), c, scale=16.0, iters=0)
    assert kind == 1 and np.abs(Ag[:, 2] - V[:2].mean(0)).max() < 1e-12
    Ag, kind = oracle.gm_fit(P, V, np.zeros(n, np.uint8), c, scale=16.0)
    assert kind == 0 and not Ag.any()
    # a pure translation of every sample is recovered exactly
    Ag, kind = oracle.gm_fit(P, np.tile([7.25, -3.5], (n, 1)), np.ones(n, np.uint8), c, scale=16.0)
    assert np.abs(Ag - [[0, 0, 7.25], [0, 0, -3.5]]).max() < 1e-10


def _occluder_pair(t=(2, 1)):
    """Low-contrast texture (values within 20 of each other, so every cross arm spans it) and a
    brighter 12 x 12 block (beyond tau from all of it); everything moves by the integer t, but in
    the second frame the block's inner 10 x 10 changes by up to +-15 (its one-pixel ring, and so
    every gradient at its edge, stays as it was)."""
    W, H, margin = 96, 96, 16
    rng = np.random.default_rng(11)
    C = np.rint(95.0 + 20.0 * synth.smoothed_noise(rng, W + 2 * margin, H + 2 * margin, 2.0) / 255.0)
    C[margin + 50:margin + 62, margin + 50:margin + 62] = 141.0
    tx, ty = t
    I0 = C[margin:margin + H, margin:margin + W].copy()
    I1 = C[margin - ty:margin - ty + H, margin - tx:margin - tx + W].copy()
    I1[51 + ty:61 + ty, 51 + tx:61 + tx] += np.rint(np.random.default_rng(3).uniform(-15, 15, (10, 10)))
    return I0.astype(np.uint8), I1.astype(np.uint8)


def _template_ext(I, p, s):
    """The patch the tracker decides the cross region on: pixels at floor(p) + k, k in [-r-1, r+1]^2,
    border replicated."""
    r = s // 2
    H, W = I.shape
    ys = np.clip(int(np.floor(p[1])) + np.arange(-r - 1, r + 2), 0, H - 1)
    xs = np.clip(int(np.floor(p[0])) + np.arange(-r - 1, r + 2), 0, W - 1)
    return I.astype(np.float64)[np.ix_(ys, xs)]


def test_cross_support_excludes_a_changing_block_exactly():
    I0, I1 = _occluder_pair()
    P = np.array([[48.0, 48.0], [47.5, 49.25], [50.3, 47.1], [45.6, 44.2]])
    for p in P:  # the block (and every sample whose gradient stencil reaches it) is outside
        Tx = _template_ext(I0, p, 21)
        m = oracle.cross_mask(Tx).astype(bool)
        assert 150 < m.sum() < 441
        near = np.zeros((21, 21), bool)
        for dy, dx in ((1, 1), (0, 1), (2, 1), (1, 0), (1, 2)):
            near |= Tx[dy:dy + 21, dx:dx + 21] >= 141.0 - 1e-9
        assert near.any() and not (m & near).any()
    # with the cross-based support only the texture is matched: its residual vanishes at the true
    # shift (the texture is faint, so the trackability floor is lowered for this case)
    kw = dict(eps_fine=1e-11, min_eig=0.1)
    f, st = oracle.track(I0, I1, P, 1, 21, 300, cross=True, **kw)
    assert np.all(st == 0)
    assert np.abs(f - [2.0, 1.0]).max() < 1e-9
    # the square support also sees the block's changed interior: samples straddling its ring
    # carry a gradient and a residual of up to 15 (inside the robust band), which pull the
    # fractional-position points off the true shift
    f2, st2 = oracle.track(I0, I1, P, 1, 21, 300, **kw)
    assert np.abs(f2[1:] - [2.0, 1.0]).max(1).min() > 1e-3


def test_cross_support_of_a_uniform_texture_is_the_square():
    # texture within tau everywhere: the support is the full window and tracking is unchanged
    I0, I1 = _canvas_uint8(seed=2, amp=20.0)
    P = np.array([[40.3, 37.8], [55.0, 41.5], [33.2, 60.7]])
    for p in P:
        assert oracle.cross_mask(_template_ext(I0, p, 15)).all()
    a = oracle.track(I0, I1, P, 2, 15, 20, cross=True, return_iters=True, min_eig=0.1)
    b = oracle.track(I0, I1, P, 2, 15, 20, return_iters=True, min_eig=0.1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def _canvas_uint8(seed, amp, t=(3, -1), W=96, H=96, m=16):
    rng = np.random.default_rng(seed)
    C = np.rint(100.0 + amp * synth.smoothed_noise(rng, W + 2 * m, H + 2 * m, 2.0) / 255.0)
    I0 = C[m:m + H, m:m + W].copy()
    I1 = C[m - t[1]:m - t[1] + H, m - t[0]:m - t[0] + W].copy()
    return I0.astype(np.uint8), I1.astype(np.uint8)


def test_gm_prior_starts_at_the_fitted_motion():
    # one level: the prior pass is the level itself; it finds the integer shift (to within its
    # stopping step), the fit is that translation, and the tracking proper starts on it and stops
    # after one step
    W, H, t = 120, 90, (3, -2)
    rng = np.random.default_rng(9)
    C = np.rint(synth.smoothed_noise(rng, W + 40, H + 40, 2.0)).astype(np.uint8)
    I0 = C[20:20 + H, 20:20 + W].copy()
    I1 = C[20 - t[1]:20 - t[1] + H, 20 - t[0]:20 - t[0] + W].copy()
    g = np.random.default_rng(1)
    P = np.stack([g.uniform(12, W - 13, 150), g.uniform(12, H - 13, 150)], 1)
    f, st, its, A = oracle.track(I0, I1, P, 1, 9, 30, gm=True, return_iters=True, return_gm=True)
    assert np.abs(A - [[0, 0, t[0]], [0, 0, t[1]]]).max() < 1e-5
    ok = st == 0
    assert ok.mean() > 0.95
    assert np.abs(f[ok] - t).max() < 1e-6
    assert np.all(its[ok, 0] == 1)
    f0, st0, its0 = oracle.track(I0, I1, P, 1, 9, 30, return_iters=True)
    assert its0[st0 == 0, 0].mean() > 2


def test_gm_prior_carries_points_that_are_flat_at_coarse_levels():
    # left half: coarse texture that survives the pyramid; right half: fine texture that the
    # pyramid smooths flat.  A shift of (6, 4) px is found on the coarse half at the top level;
    # without a prior the fine half starts from zero at full resolution and loses the match, with
    # it the fine half starts on the fitted shift and converges exactly.
    W, H, t, m = 160, 96, (6, 4), 24
    rng = np.random.default_rng(4)
    coarse = synth.smoothed_noise(rng, W + 2 * m, H + 2 * m, 4.0)
    fine = 128.0 + 0.35 * (synth.smoothed_noise(rng, W + 2 * m, H + 2 * m, 0.7) - 128.0)
    C = np.where(np.arange(W + 2 * m)[None, :] < (W + 2 * m) // 2, coarse, fine)
    C = np.rint(C).astype(np.uint8)
    I0 = C[m:m + H, m:m + W].copy()
    I1 = C[m - t[1]:m - t[1] + H, m - t[0]:m - t[0] + W].copy()
    g = np.random.default_rng(2)
    right = np.stack([g.uniform(W // 2 + 14, W - 14, 120), g.uniform(14, H - 14, 120)], 1)
    left = np.stack([g.uniform(14, W // 2 - 14, 120), g.uniform(14, H - 14, 120)], 1)
    P = np.concatenate([left, right])
    kw = dict(eps_fine=1e-10)  # exact shifts: converge far below the default step test
    f, st, A = oracle.track(I0, I1, P, 3, 9, 100, gm=True, return_gm=True, **kw)
    assert np.abs(A[:, 2] - t).max() < 0.25  # the top-level pass stops within eps_coarse (0.04 px here)
    good = (st == 0) & (np.abs(f - t).max(1) < 1e-6)
    f0, st0 = oracle.track(I0, I1, P, 3, 9, 100, **kw)
    good0 = (st0 == 0) & (np.abs(f0 - t).max(1) < 1e-6)
    n = len(left)
    print(f"right half exact: with prior {good[n:].mean():.2f}, without {good0[n:].mean():.2f}")
    assert good[n:].mean() > 0.9
    assert good0[n:].mean() < 0.3
    assert good[:n].mean() > 0.7


def test_cross_support_trackability_is_normalised_by_the_support_size():
    # an 11 x 11 textured patch on a dark frame: the cross support is the patch (eroded by the
    # gradient stencil), a fraction of the 21 x 21 window.  Its smallest gradient eigenvalue per
    # support pixel passes a trackability floor that the same eigenvalue per window pixel would not.
    W = H = 96
    rng = np.random.default_rng(6)
    I0 = np.full((H, W), 30.0)
    I0[43:54, 43:54] = np.rint(100.0 + 20.0 * synth.smoothed_noise(rng, 11, 11, 1.0) / 255.0)
    I1 = np.roll(I0, 1, axis=1)
    p = np.array([[48.0, 48.0]])
    T = I0[37:60, 37:60]  # integer position: the template extension is the image itself
    m = oracle.cross_mask(T).astype(bool)
    gx = 0.5 * (T[1:-1, 2:] - T[1:-1, :-2])
    gy = 0.5 * (T[2:, 1:-1] - T[:-2, 1:-1])
    G = np.array([[np.sum(gx[m] ** 2), np.sum(gx[m] * gy[m])], [np.sum(gx[m] * gy[m]), np.sum(gy[m] ** 2)]])
    lam = np.linalg.eigvalsh(G)[0]
    assert 40 < m.sum() < 150
    floor = np.sqrt(lam / m.sum() * lam / 441.0)  # between the two normalisations
    f, st = oracle.track(I0.astype(np.uint8), I1.astype(np.uint8), p, 1, 21, 30, cross=True, min_eig=floor)
    assert st[0] == 0 and abs(f[0, 0] - 1.0) < 1e-3
