"""Pins of the FP64 oracle's DeGraF detection (DeGraF-Flow Section 2, "Point detection",
Eq. (1)-(2) and the selection rule) against closed forms, invariants and exact brute force."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from brute import degraf_window_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = v
    return vals


@pytest.mark.parametrize("W,H,w,d", [(256, 128, 9, 8), (1242, 375, 9, 5), (1242, 375, 3, 9),
                                     (2048, 1024, 9, 2), (9, 9, 9, 1), (8, 20, 9, 3), (20, 8, 9, 3),
                                     (10, 10, 3, 100), (12, 10, 5, 4)])
def test_count_formula(W, H, w, d):
    # windows fully inside the image, origins at multiples of the step from (0, 0)
    nx = len(range(0, W - w + 1, d)) if W >= w else 0
    ny = len(range(0, H - w + 1, d)) if H >= w else 0
    assert oracle.detect_count(W, H, w, d) == nx * ny


def test_known_counts():
    assert oracle.detect_count(256, 128, 9, 8) == 465
    assert oracle.detect_count(1242, 375, 9, 5) == 18278
    assert oracle.detect_count(1242, 375, 3, 9) == 5796
    assert oracle.detect_count(2048, 1024, 9, 2) == 518160
    assert oracle.detect_count(128, 64, 9, 6) == 200


def test_ramp_worked_example_golden():
    g = _golden("degraf_ramp_w9.txt")
    img = np.tile((10 * np.arange(9)).astype(np.uint8), (9, 1))
    S = oracle.window_sums(img, 0, 0, 9, 9)
    assert S[0] == int(g["S_pos"]) and S[3] == int(g["S_neg"]) and S[6] == int(g["m"])
    pts, sel, resp = oracle.detect(img, 9, 1)
    assert pts.shape == (1, 2)
    assert sel[0] == (1 if g["selected"] == "neg" else 0)
    cneg = int(g["cneg_col_num"]) / int(g["cneg_col_den"])
    cpos = int(g["cpos_col_num"]) / int(g["cpos_col_den"])
    assert abs(pts[0, 0] - cneg) < 1e-12
    assert abs(pts[0, 1] - float(g["row"])) < 1e-12
    assert abs(resp[0] - abs(cpos - cneg)) < 1e-12


@pytest.mark.parametrize("a,b,w", [(0, 10, 9), (20, 3, 9), (5, 7, 5), (100, 1, 11), (0, 1, 3)])
def test_ramp_closed_form(a, b, w):
    # window of I = a + b*j:  C_pos col = (a w(w-1)/2 + b (w-1)w(2w-1)/6) / (a w + b w(w-1)/2)
    img = (a + b * np.arange(w))[None, :].repeat(w, 0).astype(np.uint8)
    num = Fraction(a * w * (w - 1), 2) + Fraction(b * (w - 1) * w * (2 * w - 1), 6)
    den = a * w + Fraction(b * w * (w - 1), 2)
    cpos = num / den
    m = a + b * (w - 1)
    # negative weights 1 + m - I = (1 + b(w-1)) - b j : the mirrored ramp
    a2, b2 = 1 + b * (w - 1), -b
    num2 = Fraction(a2 * w * (w - 1), 2) + Fraction(b2 * (w - 1) * w * (2 * w - 1), 6)
    den2 = a2 * w + Fraction(b2 * w * (w - 1), 2)
    cneg = num2 / den2
    S = oracle.window_sums(img, 0, 0, w, w)
    assert S[0] == w * den and S[3] == w * den2 and S[6] == m
    pts, sel, resp = oracle.detect(img, w, 1)
    neg = w * den2 > w * den
    assert sel[0] == int(neg)
    assert abs(pts[0, 0] - float(cneg if neg else cpos)) < 1e-12
    assert abs(pts[0, 1] - (w - 1) / 2) < 1e-12
    # transposed ramp: the two coordinates swap
    ptsT, selT, _ = oracle.detect(np.ascontiguousarray(img.T), w, 1)
    assert selT[0] == sel[0]
    assert abs(ptsT[0, 1] - pts[0, 0]) < 1e-12 and abs(ptsT[0, 0] - pts[0, 1]) < 1e-12


@pytest.mark.parametrize("c", [0, 1, 77, 254, 255])
def test_constant_image(c):
    w, d = 9, 4
    img = np.full((31, 40), c, np.uint8)
    pts, sel, resp = oracle.detect(img, w, d)
    nx = (40 - w) // d + 1
    n = np.arange(len(pts))
    x0, y0 = (n % nx) * d, (n // nx) * d
    assert np.array_equal(pts[:, 0], x0 + (w - 1) / 2)
    assert np.array_equal(pts[:, 1], y0 + (w - 1) / 2)
    assert np.all(resp == 0.0)
    # S_neg = w*h (all weights 1) beats S_pos = c*w*h only when c = 0
    assert np.all(sel == (1 if c == 0 else 0))


def _random_img(rng, W, H):
    return rng.integers(0, 256, size=(H, W), dtype=np.uint8)


@pytest.mark.parametrize("m_mode", [0, 1])
def test_collinearity_and_sums_invariant(m_mode):
    # I + (1 + m - I) = 1 + m per pixel, so the moment sums add up to (1+m) times those of a
    # constant window, exactly in integers.
    rng = np.random.default_rng(5)
    img = _random_img(rng, 30, 25)
    for (x0, y0, w, h) in [(0, 0, 9, 9), (3, 7, 5, 5), (10, 2, 7, 11), (1, 1, 1, 1)]:
        S = oracle.window_sums(img, x0, y0, w, h, m_mode)
        m = S[6]
        assert S[0] + S[3] == (1 + m) * w * h
        assert S[1] + S[4] == (1 + m) * w * h * (h - 1) // 2
        assert S[2] + S[5] == (1 + m) * h * w * (w - 1) // 2


def test_offset_and_gain_invariance():
    rng = np.random.default_rng(6)
    base = rng.integers(0, 100, size=(20, 20)).astype(np.int64)
    w = 9
    S1 = oracle.window_sums(base.astype(np.uint8), 2, 3, w, w)
    # offset: I + c leaves the negative centroid unchanged (m moves with I)
    S2 = oracle.window_sums((base + 120).astype(np.uint8), 2, 3, w, w)
    assert Fraction(S1[5], S1[3]) == Fraction(S2[5], S2[3])
    assert Fraction(S1[4], S1[3]) == Fraction(S2[4], S2[3])
    # gain: g * I leaves the positive centroid unchanged
    S3 = oracle.window_sums((base * 2).astype(np.uint8), 2, 3, w, w)
    assert Fraction(S1[2], S1[0]) == Fraction(S3[2], S3[0])
    assert Fraction(S1[1], S1[0]) == Fraction(S3[1], S3[0])


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_fraction(seed):
    rng = np.random.default_rng(100 + seed)
    W, H = int(rng.integers(5, 13)), int(rng.integers(5, 11))
    w = int(rng.integers(1, 6))
    d = int(rng.integers(1, 5))
    img = _random_img(rng, W, H)
    if seed % 3 == 0:  # include flat and dark windows
        img[: H // 2, : W // 2] = 0
    if seed % 4 == 1:
        img[H // 2:, :] = 200
    for m_mode in (0, 1):
        pts, sel, resp = oracle.detect(img, w, d, m_mode=m_mode)
        nx = (W - w) // d + 1
        assert len(pts) == oracle.detect_count(W, H, w, d)
        for n in range(len(pts)):
            x0, y0 = (n % nx) * d, (n // nx) * d
            win = img[y0:y0 + w, x0:x0 + w].astype(int).tolist()
            ex = degraf_window_exact(win, m_mode)
            assert sel[n] == int(ex["neg"])
            assert abs(pts[n, 0] - (x0 + float(ex["point"][0]))) <= 1e-12
            assert abs(pts[n, 1] - (y0 + float(ex["point"][1]))) <= 1e-12
            cp = ex["C_pos"] if ex["C_pos"] is not None else (Fraction(w - 1, 2), Fraction(w - 1, 2))
            rr = float(((cp[0] - ex["C_neg"][0]) ** 2 + (cp[1] - ex["C_neg"][1]) ** 2)) ** 0.5
            assert abs(resp[n] - rr) <= 1e-12


def test_points_inside_their_windows():
    rng = np.random.default_rng(7)
    img = _random_img(rng, 97, 61)
    w, d = 9, 5
    pts, _, _ = oracle.detect(img, w, d)
    nx = (97 - w) // d + 1
    n = np.arange(len(pts))
    x0, y0 = (n % nx) * d, (n // nx) * d
    assert np.all(pts[:, 0] >= x0) and np.all(pts[:, 0] <= x0 + w - 1)
    assert np.all(pts[:, 1] >= y0) and np.all(pts[:, 1] <= y0 + w - 1)


def test_shift_transpose_flip():
    rng = np.random.default_rng(8)
    w, d = 9, 5
    W, H = 9 + 5 * 12, 9 + 5 * 8  # (W - w) and (H - w) divisible by d
    img = _random_img(rng, W, H)
    pts, sel, _ = oracle.detect(img, w, d)
    nx, ny = (W - w) // d + 1, (H - w) // d + 1
    P = pts.reshape(ny, nx, 2)
    S = sel.reshape(ny, nx)
    # shift: crop by (a d, b d) -> interior windows are the same windows, moved
    a, b = 2, 3
    pts2, sel2, _ = oracle.detect(img[b * d:, a * d:], w, d)
    P2 = pts2.reshape(ny - b, nx - a, 2)
    assert np.allclose(P2 + np.array([a * d, b * d]), P[b:, a:], atol=1e-12, rtol=0)
    assert np.array_equal(sel2.reshape(ny - b, nx - a), S[b:, a:])
    # transpose: window grid transposes, coordinates swap
    ptsT, selT, _ = oracle.detect(np.ascontiguousarray(img.T), w, d)
    PT = ptsT.reshape(nx, ny, 2)
    assert np.allclose(PT[..., ::-1], P.transpose(1, 0, 2), atol=1e-12, rtol=0)
    assert np.array_equal(selT.reshape(nx, ny), S.T)
    # horizontal flip mirrors x about (W - 1) / 2 and reverses the window columns
    ptsF, selF, _ = oracle.detect(np.ascontiguousarray(img[:, ::-1]), w, d)
    PF = ptsF.reshape(ny, nx, 2)[:, ::-1]
    assert np.allclose(PF[..., 0], (W - 1) - P[..., 0], atol=1e-12, rtol=0)
    assert np.allclose(PF[..., 1], P[..., 1], atol=1e-12, rtol=0)
    assert np.array_equal(selF.reshape(ny, nx)[:, ::-1], S)


def test_empty_cases():
    img = np.zeros((5, 5), np.uint8)
    pts, sel, resp = oracle.detect(img, 9, 2)
    assert pts.shape == (0, 2)
