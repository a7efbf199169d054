"""GPU parity of DeGraF detection (HIP kernel through the C ABI) against the FP64 oracle.
Point count and window order are exact by construction; the centroid selection bit must be
bit-exact (integer comparison); positions and responses within 1e-3 px."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import _lib, synth

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _compare(img_np, window, stride, gpu_img=None):
    t = gpu_img if gpu_img is not None else torch.from_numpy(img_np).cuda()
    pts, sel, resp = dgf.detect(t, window, stride, return_sel=True, return_response=True)
    torch.cuda.synchronize()
    opts, osel, oresp = oracle.detect(img_np, window, stride)
    assert pts.shape[0] == opts.shape[0] == oracle.detect_count(img_np.shape[1], img_np.shape[0], window, stride)
    if len(opts) == 0:
        return
    assert np.array_equal(sel.cpu().numpy(), osel)
    err = np.abs(pts.cpu().numpy().astype(np.float64) - opts).max()
    assert err <= TOL, err
    assert np.abs(resp.cpu().numpy() - oresp).max() <= TOL


def test_translation_256x128():
    I0, _, _ = synth.translation_256x128()
    _compare(I0, 9, 8)


def test_driving_1242x375_stride5_and_paper_params():
    I0, _, _, _ = synth.driving_1242x375()
    _compare(I0, 9, 5)
    _compare(I0, 3, 9)  # the paper's DeGraF setting w = h = 3, delta = 9


def test_density_2048x1024_stride2():
    I0, _, _, _ = synth.density_2048x1024(0)
    _compare(I0, 9, 2)


@pytest.mark.parametrize("seed", range(10))
def test_random_ragged(seed):
    rng = np.random.default_rng(seed)
    W, H = int(rng.integers(9, 300)), int(rng.integers(9, 200))
    window = int(rng.integers(1, min(W, H, 24) + 1))
    stride = int(rng.integers(1, 13))
    img = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    if seed % 2:
        img[: H // 3] = 0
        img[-H // 4:] = 255
    _compare(img, window, stride)


def test_window_equals_image_and_empty():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(20, 20), dtype=np.uint8)
    _compare(img, 20, 1)
    _compare(img, 21, 1)  # image smaller than the window: no points


def test_large_window_direct_path():
    I0, _, _, _ = synth.driving_1242x375()
    _compare(I0, 128, 100)
    _compare(I0, 100, 3)


@pytest.mark.parametrize("value", [0, 255])
def test_flat_images(value):
    _compare(np.full((64, 80), value, np.uint8), 9, 4)


def test_pitched_input():
    rng = np.random.default_rng(4)
    big = rng.integers(0, 256, size=(120, 300), dtype=np.uint8)
    view = torch.from_numpy(big).cuda()[:, 13:213]  # pitch 300, width 200
    _compare(np.ascontiguousarray(big[:, 13:213]), 9, 5, gpu_img=view)


def test_capacity_and_argument_errors():
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    im = _lib.DgfImage(img.data_ptr(), 64, 64, 64, _lib.DGF_U8)
    out = torch.empty((10, 2), dtype=torch.float32, device="cuda")
    L = _lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.dgf_detect(ctypes.byref(im), 9, 8, ctypes.c_void_p(out.data_ptr()), None, None, 10, s) == -2
    assert L.dgf_detect(ctypes.byref(im), 0, 8, ctypes.c_void_p(out.data_ptr()), None, None, 10, s) == -1
    assert L.dgf_detect(ctypes.byref(im), 200, 8, ctypes.c_void_p(out.data_ptr()), None, None, 10, s) == -1
