"""GPU tests of the batched form (one plan for many pairs of uneven size and point count):
its output must be bit-identical to per-pair plain detect + track calls with the same launch
shape, and graph replays must reproduce the eager run."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth
from parity import compare_tracks

pytestmark = pytest.mark.gpu

SIZES = [(1242, 375), (640, 480), (320, 240), (77, 41), (8, 8), (1224, 370)]
STRIDES = [5, 8, 3, 4, 2, 7]


def _pairs(n, max_disp=60.0):
    out = []
    for i in range(n):
        W, H = SIZES[i % len(SIZES)]
        if W < 32:
            I0 = np.random.default_rng(i).integers(0, 256, size=(H, W), dtype=np.uint8)
            I1 = I0.copy()
        else:
            I0, I1, _, _ = synth.layered_pair(W, H, seed=100 + i, max_disp=max_disp * W / 1242.0)
        out.append((torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), 9, STRIDES[i % len(STRIDES)]))
    return out


def _plain(pairs, levels, support, iters):
    pts, flow, st = [], [], []
    for a, b, w, d in pairs:
        p = dgf.detect(a, w, d)
        f, s = dgf.track(a, b, p, levels, support, iters)
        pts.append(p)
        flow.append(f)
        st.append(s)
    return torch.cat(pts), torch.cat(flow), torch.cat(st)


@pytest.mark.parametrize("levels,support,iters", [(5, 21, 20), (3, 9, 10)])
def test_batched_equals_plain(levels, support, iters):
    pairs = _pairs(12)
    plan = dgf.Batch(pairs, levels, support, iters)
    P, F, S = plan.run()
    p, f, s = _plain(pairs, levels, support, iters)
    torch.cuda.synchronize()
    assert plan.num_points == p.shape[0]
    assert plan.offsets[-1] == p.shape[0]
    assert torch.equal(P, p)
    assert torch.equal(S, s)
    fin = torch.isfinite(f)
    assert torch.equal(torch.isfinite(F), fin)
    assert torch.equal(F[fin], f[fin])
    plan.close()


def test_graph_replay_matches_eager():
    pairs = _pairs(8)
    plan = dgf.Batch(pairs, 5, 21, 20)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        P0, F0, S0 = [t.clone() for t in plan.run()]
        plan.capture()
    torch.cuda.synchronize()
    for rep in range(4):
        with torch.cuda.stream(side):
            plan.points.zero_()
            plan.flow.zero_()
            plan.status.fill_(255)
            plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.points, P0), rep
        assert torch.equal(plan.status, S0), rep
        fin = torch.isfinite(F0)
        assert torch.equal(plan.flow[fin], F0[fin]), rep
        # eager work on the default stream between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum().item()
    plan.close()


def test_batched_pair_vs_oracle_sample():
    pairs = _pairs(3)
    plan = dgf.Batch(pairs, 4, 15, 15)
    P = plan.front().cpu().numpy()
    frames = [(a.cpu().numpy(), b.cpu().numpy()) for a, b, _, _ in pairs]
    oP = np.concatenate([oracle.detect(I0, w, d)[0] for (I0, _), (_, _, w, d) in zip(frames, pairs)])
    assert P.shape == oP.shape and np.abs(P - oP).max() <= 1e-3
    # the plan tracks the oracle's points (FP32) on its own pyramids; the oracle tracks the same
    oP = oP.astype(np.float32)
    F, S = [t.cpu().numpy() for t in plan.track(torch.from_numpy(oP).cuda())]
    for i, (I0, I1) in enumerate(frames):
        lo, hi = plan.offsets[i], plan.offsets[i + 1]
        idx = np.arange(lo, hi, 7)  # every 7th point of the pair
        of, os_ = oracle.track(I0, I1, oP[idx].astype(np.float64), 4, 15, 15)
        compare_tracks(F[idx], S[idx], of, os_, 0.999, 1e-3, label=f"batched pair {i}")
    plan.close()


def test_invalid_plans():
    a = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    f = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        dgf.Batch([(a, f, 9, 4)], 3, 9, 10)          # mixed dtypes
    with pytest.raises(RuntimeError):
        dgf.Batch([(a, a, 9, 4)], 3, 8, 10)          # even support
    with pytest.raises(RuntimeError):
        dgf.Batch([(f, f, 9, 4)], 3, 9, 10)          # float frames cannot be detected on
    empty = dgf.Batch([(a[:4, :4].contiguous(), a[:4, :4].contiguous(), 9, 4)], 3, 9, 10)
    assert empty.num_points == 0
    empty.run()
    empty.close()


def test_batched_backward_equals_per_pair_backward():
    """One adjoint launch over the plan equals dgf_track_backward pair by pair (on float copies of
    the frames, same values), up to the order of the float atomics."""
    pairs = _pairs(6, max_disp=30.0)
    plan = dgf.Batch(pairs, 4, 21, 20)
    P, F, S = plan.run()
    g = torch.Generator(device="cpu").manual_seed(7)
    dflow = torch.randn(plan.num_points, 2, generator=g).cuda()
    grad, views = plan.backward(dflow)
    torch.cuda.synchronize()
    total, off = plan.grad_layout()
    assert grad.numel() >= total and off[-1] == total
    for i, (a, b, _, _) in enumerate(pairs):
        lo, hi = plan.offsets[i], plan.offsets[i + 1]
        a32, b32 = a.float(), b.float()
        dI0, dI1 = torch.zeros_like(a32), torch.zeros_like(b32)
        if hi > lo:
            dgf.track_backward(a32, b32, P[lo:hi], 21, F[lo:hi], S[lo:hi], dflow[lo:hi], dI0, dI1)
        g0, g1 = views[i]
        for got, ref in ((g0, dI0), (g1, dI1)):
            scale = float(ref.abs().max()) + 1e-30
            assert float((got - ref).abs().max()) <= 1e-5 * scale, (i, float((got - ref).abs().max()), scale)
        if int((S[lo:hi] == 0).sum()) > 0:
            assert float(dI1.abs().max()) > 0.0
    # a second call overwrites (does not accumulate)
    grad2, _ = plan.backward(dflow, grad)
    torch.cuda.synchronize()
    assert torch.allclose(grad2[:total], grad[:total], rtol=0, atol=1e-5 * float(grad[:total].abs().max()))
    plan.close()


def test_track_batched_convenience_equals_per_pair():
    pairs = []
    for i, (W, H) in enumerate([(320, 240), (200, 150)]):
        I0, I1, _, _ = synth.layered_pair(W, H, seed=70 + i, max_disp=20.0)
        pairs.append((torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), 9, 7))
    outs = dgf.track_batched(pairs, 4, 21, 20)
    for (a, b, w, d), (P, F, S) in zip(pairs, outs):
        p = dgf.detect(a, w, d)
        f, s = dgf.track(a, b, p, 4, 21, 20)
        assert torch.equal(P, p) and torch.equal(S, s)
        fin = torch.isfinite(f)
        assert torch.equal(F[fin], f[fin])


def test_front_then_track_equals_run():
    pairs = _pairs(6)
    plan = dgf.Batch(pairs, 4, 21, 20)
    P, F, S = [t.clone() for t in plan.run()]
    plan.points.zero_()
    plan.flow.zero_()
    plan.status.fill_(255)
    plan.front()
    plan.track()
    torch.cuda.synchronize()
    assert torch.equal(plan.points, P) and torch.equal(plan.status, S)
    fin = torch.isfinite(F)
    assert torch.equal(torch.isfinite(plan.flow), fin) and torch.equal(plan.flow[fin], F[fin])
    plan.close()


def _device_level(addr, pitch, w, h):
    """Copy a uint8 device image (address, row pitch) into a new [h, w] tensor (hipMemcpy2D)."""
    import ctypes
    # the HIP runtime this process already uses (torch's), not a second copy
    with open("/proc/self/maps") as f:
        path = next(ln.split()[-1] for ln in f if "libamdhip64" in ln)
    hip = ctypes.CDLL(path)
    out = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc = hip.hipMemcpy2D(ctypes.c_void_p(out.data_ptr()), ctypes.c_size_t(w), ctypes.c_void_p(addr),
                         ctypes.c_size_t(pitch), ctypes.c_size_t(w), ctypes.c_size_t(h), 3)  # device to device
    assert rc == 0
    return out


@pytest.mark.parametrize("seed", range(12))
def test_plan_pyramids_equal_per_frame_pyramids(seed):
    # every level of every frame the batched front end builds (level 1 beside detection, the
    # coarser levels in one launch) equals dgf_pyramid of that frame, bit for bit
    rng = np.random.default_rng(1000 + seed)
    pairs = []
    for _ in range(int(rng.integers(1, 9))):
        W, H = int(rng.integers(8, 2100)), int(rng.integers(8, 1100))
        a = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        b = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        pairs.append((torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), 9, int(rng.integers(2, 9))))
    levels = int(rng.integers(2, 9))
    plan = dgf.Batch(pairs, levels, 9, 10)
    for rep in range(2):  # a second front reuses the counters the first one left
        plan.front()
        torch.cuda.synchronize()
        for i, (a, b, _, _) in enumerate(pairs):
            for f, img in enumerate((a, b)):
                ref = dgf.pyramid(img, levels)
                for l in range(1, levels):
                    got = _device_level(*plan.level(i, f, l))
                    assert torch.equal(got, ref[l]), (seed, rep, i, f, l, tuple(img.shape))
    with pytest.raises(RuntimeError):
        plan.level(len(pairs), 0, 1)
    plan.close()
