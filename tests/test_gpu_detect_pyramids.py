"""dgf_detect_pyramids (detection beside the first pyramid-chain launch) against the two separate
calls, dgf_detect and dgf_track_pyramids, through the C ABI: points, selections and responses
bit-identical, every pyramid level of both frames byte-identical, for ragged grids, window sizes
up to the largest the fused launch stages, one and two chain launches, and the fallbacks (one
level, no points, a detection tile too large to fuse)."""
import numpy as np
import pytest
import torch

import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth

pytestmark = pytest.mark.gpu


def _both(I0, I1, window, stride, levels):
    a, b = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    H, W = I0.shape
    n = dgf.detect_count(W, H, window, stride)
    nb = dgf.track_workspace_bytes(W, H, levels, 0)
    ws1 = torch.zeros(max(nb, 1), dtype=torch.uint8, device="cuda")
    ws2 = torch.full((max(nb, 1),), 7, dtype=torch.uint8, device="cuda")
    P1, s1, r1 = dgf.detect(a, window, stride, return_sel=True, return_response=True)
    dgf.track_pyramids(a, b, levels, ws1)
    P2 = torch.full((n, 2), float("nan"), dtype=torch.float32, device="cuda")
    s2 = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
    r2 = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    dgf.detect_pyramids(a, b, window, stride, levels, ws2, P2, s2, r2)
    torch.cuda.synchronize()
    print(f"{W}x{H} w{window} d{stride} L{levels}: n={n}", flush=True)
    assert torch.equal(P2.view(torch.int32), P1.view(torch.int32))
    assert torch.equal(s2, s1)
    assert torch.equal(r2.view(torch.int32), r1.view(torch.int32))
    # every coarser level of both frames (I0's pyramid, then I1's, in the workspace)
    total, off, pit = dgf.pyramid_layout(W, H, levels, 0)
    Wl, Hl = W, H
    for l in range(1, levels):
        Wl, Hl = (Wl + 1) // 2, (Hl + 1) // 2
        for f in range(2):
            o = f * total + off[l]
            v1 = ws1[o:o + pit[l] * Hl].view(Hl, pit[l])[:, :Wl]
            v2 = ws2[o:o + pit[l] * Hl].view(Hl, pit[l])[:, :Wl]
            assert torch.equal(v1, v2), (l, f)
    return n


def test_driving_1242x375_benchmark_shape():
    I0, I1, _, _ = synth.driving_1242x375()
    assert _both(I0, I1, 9, 5, 5) == 18278


@pytest.mark.parametrize("W,H,window,stride,levels", [
    (333, 251, 9, 7, 4), (640, 480, 9, 3, 6), (97, 61, 1, 1, 3), (257, 129, 2, 2, 2), (301, 257, 15, 4, 5),
    (1024, 700, 64, 17, 7), (700, 500, 21, 10, 12), (53, 47, 31, 6, 3)])
def test_sizes_windows_levels(W, H, window, stride, levels):
    I0, I1, _, _ = synth.layered_pair(W, H, seed=window + levels, max_disp=10.0)
    _both(I0, I1, window, stride, levels)


def test_fallbacks():
    I0, I1, _, _ = synth.layered_pair(400, 300, seed=1, max_disp=5.0)
    _both(I0, I1, 9, 5, 1)        # one level: detection alone
    _both(I0, I1, 128, 60, 4)     # tile of 1028 x 1028 bytes: two launches
    _both(I0[:8, :8].copy(), I1[:8, :8].copy(), 9, 1, 3)  # no points: pyramids alone


def test_odd_pitch_misaligned_frames_through_tracking():
    # frames as views with an odd row pitch (1249 bytes) and bases 3 and 6 bytes into their
    # buffers, so every image row starts at a different dword alignment; detection beside the
    # pyramids and tracking on them must equal the same frames stored contiguously, bit for bit
    I0, I1, _, _ = synth.driving_1242x375()
    H, W = I0.shape
    big0 = np.zeros((H, W + 7), np.uint8)
    big1 = np.zeros((H, W + 7), np.uint8)
    big0[:, 3:3 + W] = I0
    big1[:, 6:6 + W] = I1
    v0, v1 = torch.from_numpy(big0).cuda()[:, 3:3 + W], torch.from_numpy(big1).cuda()[:, 6:6 + W]
    c0, c1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    assert v0.stride(0) == W + 7 and v0.data_ptr() % 4 == 3
    n = dgf.detect_count(W, H, 9, 5)
    out = []
    for a, b in ((c0, c1), (v0, v1)):
        ws = torch.empty(dgf.track_workspace_bytes(W, H, 5, 0), dtype=torch.uint8, device="cuda")
        P = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        F = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        S = torch.empty(n, dtype=torch.uint8, device="cuda")
        dgf.detect_pyramids(a, b, 9, 5, 5, ws, P)
        dgf.track_run(a, b, P, 5, 21, 20, ws, F, S)
        torch.cuda.synchronize()
        out.append((P, F, S))
    (P1, F1, S1), (P2, F2, S2) = out
    assert torch.equal(P1.view(torch.int32), P2.view(torch.int32))
    assert torch.equal(F1.view(torch.int32), F2.view(torch.int32))
    assert torch.equal(S1, S2)
