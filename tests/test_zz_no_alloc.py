"""dgf_track_static (tracking with the pyramids in the library's static per-GPU scratch array, no
workspace argument) against dgf_track with a caller workspace: the same kernels and launch shape
must give bit-identical flow, status, iteration counts and illumination parameters.  Two calls in
a row, the second on a smaller pair, so the second must not read anything the first left in the
shared array."""
import numpy as np
import pytest
import torch

import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _pair(I0, I1):
    return torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()


def _both(t0, t1, L, s, iters, window, stride, opts=None):
    pts = dgf.detect(t0, window, stride)
    print(f"track_static: {tuple(t0.shape)} {t0.dtype} L={L} s={s} iters={iters} n={pts.shape[0]} "
          f"illum={bool(opts and opts.illum)}", flush=True)
    ill = bool(opts and opts.illum)
    ref = dgf.track(t0, t1, pts, L, s, iters, opts=opts, return_iters=True, return_illum=ill)
    got = dgf.api.track_static(t0, t1, pts, L, s, iters, opts=opts, return_iters=True, return_illum=ill)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert a.shape == b.shape
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), np.abs(a.astype(np.float64) - b).max()
    st = got[1].cpu().numpy()
    assert (st == 0).sum() > 0
    return st


def test_static_matches_workspace_two_calls_second_smaller():
    big = _pair(*synth.driving_1242x375()[:2])
    small = _pair(*synth.translation_256x128()[:2])
    _both(*big, 5, 21, 20, 9, 5)
    st = _both(*small, 3, 9, 10, 9, 8)
    assert np.mean(st == 0) > 0.95


def test_static_float_frames_and_illumination_model():
    I0, I1, _ = synth.translation_f32_1242x375()
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    # detection runs on the rounded uint8 copy of a float frame
    u0 = torch.from_numpy(np.clip(np.rint(I0), 0, 255).astype(np.uint8)).cuda()
    pts = dgf.detect(u0, 9, 8)
    ref = dgf.track(t0, t1, pts, 3, 9, 10, return_iters=True)
    got = dgf.api.track_static(t0, t1, pts, 3, 9, 10, return_iters=True)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    g0, g1 = _pair(*synth.driving_1242x375()[:2])
    g1 = torch.clamp(g1.float() * 1.15 - 12, 0, 255).round().to(torch.uint8)
    _both(g0, g1, 5, 21, 20, 9, 5, opts=dgf.TrackOpts(illum=True))


def test_static_rejects_oversized_input_without_launching():
    t = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
    pts = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.DgfError) as e:
        dgf.api.track_static(t, t, pts, 3, 9, 10)
    assert e.value.code == _lib.DGF_ERR_SCRATCH
    # the library still works after the rejection
    test_static_matches_workspace_two_calls_second_smaller()
