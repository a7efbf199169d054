"""Pins of the oracle's image pyramid (binomial 5-tap, replicated border, half-size levels)
against scipy.ndimage and polynomial invariants."""
import numpy as np
import pytest

import oracle
from brute import pyr_down_scipy


@pytest.mark.parametrize("W,H", [(1, 1), (2, 3), (5, 4), (17, 9), (256, 128), (1242, 375), (13, 64)])
def test_u8_matches_scipy(W, H):
    rng = np.random.default_rng(W * 1000 + H)
    img = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    lv = oracle.pyramid(img, 4)
    cur = img
    for l in range(1, 4):
        cur = pyr_down_scipy(cur)
        assert lv[l].shape == cur.shape
        assert np.array_equal(lv[l], cur)


@pytest.mark.parametrize("W,H", [(3, 2), (17, 9), (256, 128), (311, 94)])
def test_f64_matches_scipy(W, H):
    rng = np.random.default_rng(W + H)
    img = rng.uniform(0, 255, size=(H, W))
    lv = oracle.pyramid(img, 4)
    cur = img
    for l in range(1, 4):
        cur = pyr_down_scipy(cur)
        assert np.allclose(lv[l], cur, rtol=0, atol=1e-12)


def test_dims_ceil():
    assert oracle.pyr_dims(1242, 375, 5) == [(1242, 375), (621, 188), (311, 94), (156, 47), (78, 24)]
    assert oracle.pyr_dims(2048, 1024, 6)[-1] == (64, 32)
    assert oracle.pyr_dims(1, 1, 3) == [(1, 1), (1, 1), (1, 1)]


def test_constant_and_bilinear_span():
    c = np.full((40, 50), 93, np.uint8)
    for lv in oracle.pyramid(c, 4):
        assert np.all(lv == 93)
    # f = a + b x + c y + e x y is reproduced exactly away from the border: level 1 at (x, y)
    # equals f(2x, 2y) because the symmetric binomial kernel preserves per-axis linear terms.
    H, W = 40, 50
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    f = lambda x, y: 20 + 0.5 * x + 0.3 * y + 0.05 * x * y
    lv = oracle.pyramid(f(xx, yy), 2)
    y1, x1 = np.mgrid[1:H // 2 - 1, 1:W // 2 - 1].astype(np.float64)
    assert np.allclose(lv[1][1:H // 2 - 1, 1:W // 2 - 1], f(2 * x1, 2 * y1), atol=1e-12, rtol=0)


def test_u8_rounding_half_up():
    # a single bright pixel: level-1 value at its position is round(255 * 36 / 256) = round(35.86)
    img = np.zeros((9, 9), np.uint8)
    img[4, 4] = 255
    lv = oracle.pyramid(img, 2)
    assert lv[1][2, 2] == 36  # 255*36 = 9180; (9180 + 128) >> 8 = 36
    # neighbours one level-1 pixel away see weight 1*6 -> 255*6/256 = 5.98 -> 6
    assert lv[1][2, 1] == 6 and lv[1][1, 2] == 6
    # an exact half rounds up: pixel (2, 2) = 128 reaches level-1 pixel (0, 0) through the
    # corner tap of weight 1*1, so the sum is 128 = 0.5 * 256 -> 1
    img2 = np.zeros((9, 9), np.uint8)
    img2[2, 2] = 128
    lv2 = oracle.pyramid(img2, 2)
    assert lv2[1][0, 0] == 1
    # and through the centre tap (weight 36) of level-1 pixel (1, 1): 4608 / 256 = 18.0 -> 18
    assert lv2[1][1, 1] == 18
