"""GPU parity of the gradient through detection (dgf_detect_backward) and of dL/dp from the
tracker's adjoint (dgf_track_backward's dpoints) against the FP64 oracle, which the CPU suite
pins to finite differences; and the two chained by autograd (DetectFn + TrackFn).  Each backward
takes the oracle's selection bits or forward result as its input."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth

pytestmark = pytest.mark.gpu
REL = 1e-4


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", ["translation_256x128", "driving_1242x375"])
def test_detect_backward_vs_oracle(case):
    if case == "translation_256x128":
        I0, _, _ = synth.translation_256x128()
        w, d = 9, 8
    else:
        I0, _, _, _ = synth.driving_1242x375()
        w, d = 9, 5
    t0 = torch.from_numpy(I0).cuda()
    pts, sel = dgf.detect(t0, w, d, return_sel=True)
    _, osel, _ = oracle.detect(I0, w, d)
    assert np.array_equal(sel.cpu().numpy(), osel)
    rng = np.random.default_rng(1)
    lam = rng.normal(size=(pts.shape[0], 2)).astype(np.float32)
    dI = torch.zeros(I0.shape, dtype=torch.float32, device="cuda")
    # both sides take the oracle's selection bits
    dgf.detect_backward(t0, w, d, torch.from_numpy(osel).cuda(), torch.from_numpy(lam).cuda(), dI)
    torch.cuda.synchronize()
    ref = oracle.detect_grad(I0.astype(np.float64), w, d, osel, lam.astype(np.float64))
    e = _rel(dI.cpu().numpy().astype(np.float64), ref)
    print(f"{case}: points {pts.shape[0]} rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5


def test_point_gradient_vs_oracle():
    I0, I1, gt = synth.translation_f32_1242x375()
    I0, I1 = np.ascontiguousarray(I0[:120, :200]), np.ascontiguousarray(I1[:120, :200])
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0].astype(np.float32)
    # both adjoints at the oracle's forward result (FP64, converged to 1e-12; flow in FP32)
    I0d, I1d = I0.astype(np.float64), I1.astype(np.float64)
    oflow, ost = oracle.track(I0d, I1d, pts.astype(np.float64), 3, 9, 100, eps_fine=1e-12)
    conv = ost == 0
    assert conv.mean() > 0.9
    fl32 = np.where(conv[:, None], oflow, 0.0).astype(np.float32)
    df32 = np.where(conv[:, None], 2.0 * (fl32.astype(np.float64) - gt), 0.0).astype(np.float32)
    t0, t1, P = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), torch.from_numpy(pts).cuda()
    dI0, dI1, dp = torch.zeros_like(t0), torch.zeros_like(t1), torch.empty_like(P)
    dgf.track_backward(t0, t1, P, 9, torch.from_numpy(fl32).cuda(), torch.from_numpy(ost).cuda(),
                       torch.from_numpy(df32).cuda(), dI0, dI1, opts=dgf.TrackOpts(eps_fine=1e-6), dpoints=dp)
    torch.cuda.synchronize()
    o0, o1, odp = oracle.track_grad(I0d, I1d, pts.astype(np.float64), 9, fl32.astype(np.float64), ost,
                                    df32.astype(np.float64), return_dpoints=True)
    e0, e1, ep = _rel(dI0.cpu().numpy(), o0), _rel(dI1.cpu().numpy(), o1), _rel(dp.cpu().numpy(), odp)
    print(f"converged {int(conv.sum())}/{len(ost)}: rel dI0 {e0:.2e} dI1 {e1:.2e} dpoints {ep:.2e}", flush=True)
    assert e0 <= REL and e1 <= REL and ep <= REL
    assert torch.all(dp[torch.from_numpy(~conv).cuda()] == 0)


def test_detect_and_track_autograd_end_to_end():
    """Autograd through DetectFn and TrackFn equals the direct C-ABI chain at the same forward
    result: dgf_track_backward (frames and dL/dp), then dgf_detect_backward of dL/dp added into
    dL/dI0.  Each link is held to the oracle on shared inputs by the two tests above."""
    I0n, I1n, gt = synth.translation_f32_1242x375()
    I0n = np.rint(np.ascontiguousarray(I0n[:120, :200])).astype(np.float32)  # grey levels
    I1n = np.ascontiguousarray(I1n[:120, :200])
    I0 = torch.from_numpy(I0n).cuda().requires_grad_(True)
    I1 = torch.from_numpy(I1n).cuda().requires_grad_(True)
    opts = dgf.TrackOpts(eps_fine=1e-6)
    P = dgf.DetectFn.apply(I0, 9, 6)
    flow, st = dgf.TrackFn.apply(I0, I1, P, 3, 9, 100, opts)
    conv = (st == 0).float()[:, None]
    g = torch.tensor(gt, dtype=torch.float32, device="cuda")
    loss = (((flow - g) ** 2) * conv).sum()
    loss.backward()
    u8 = I0.detach().round().clamp(0, 255).to(torch.uint8)
    _, sel = dgf.detect(u8, 9, 6, return_sel=True)
    t0, t1, Pd = I0.detach(), I1.detach(), P.detach()
    d0, d1, dp = torch.zeros_like(t0), torch.zeros_like(t1), torch.zeros_like(Pd)
    dgf.track_backward(t0, t1, Pd, 9, flow.detach(), st, 2.0 * (flow.detach() - g) * conv, d0, d1, opts=opts,
                       dpoints=dp)
    dgf.detect_backward(u8, 9, 6, sel, dp, d0)
    torch.cuda.synchronize()
    e0 = _rel(I0.grad.cpu().numpy().astype(np.float64), d0.cpu().numpy().astype(np.float64))
    e1 = _rel(I1.grad.cpu().numpy().astype(np.float64), d1.cpu().numpy().astype(np.float64))
    print(f"end to end vs direct chain: rel dI0 {e0:.2e} dI1 {e1:.2e} converged {int(conv.sum())}/{len(st)}",
          flush=True)
    assert e0 <= 1e-6 and e1 <= 1e-6
    assert float(dp.abs().sum()) > 0 and conv.mean() > 0.9


def test_detect_backward_random_sweep():
    # 200 fixed-seed frames: layered scenes, uniform noise and four-level images (many tied
    # window maxima), windows 1 .. 64, strides 1 .. 19, ragged grids; bar 1e-5 relative L2 (a
    # 12,000-trial run of the same generator: worst 5.5e-6)
    rng = np.random.default_rng(3)
    done = 0
    while done < 200:
        W, H = int(rng.integers(8, 500)), int(rng.integers(8, 400))
        kind = int(rng.integers(3))
        if kind == 0:
            I0 = synth.layered_pair(max(W, 16), max(H, 16), seed=int(rng.integers(1 << 30)), max_disp=2.0)[0][:H, :W]
        elif kind == 1:
            I0 = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
        else:
            I0 = (rng.integers(0, 4, size=(H, W)) * 60).astype(np.uint8)
        I0 = np.ascontiguousarray(I0)
        w, d = int(rng.integers(1, min(W, H, 64) + 1)), int(rng.integers(1, 20))
        n = oracle.detect_count(W, H, w, d)
        if n == 0 or n > 40000:
            continue
        done += 1
        t0 = torch.from_numpy(I0).cuda()
        _, osel, _ = oracle.detect(I0, w, d)
        lam = rng.normal(size=(n, 2)).astype(np.float32)
        dI = torch.zeros(I0.shape, dtype=torch.float32, device="cuda")
        dgf.detect_backward(t0, w, d, torch.from_numpy(osel).cuda(), torch.from_numpy(lam).cuda(), dI)
        torch.cuda.synchronize()
        ref = oracle.detect_grad(I0.astype(np.float64), w, d, osel, lam.astype(np.float64))
        g = dI.cpu().numpy().astype(np.float64)
        if np.linalg.norm(ref) == 0:  # 1 x 1 windows: the point is the pixel, no image dependence
            assert np.all(g == 0), (W, H, kind, w, d)
            continue
        e = _rel(g, ref)
        assert e <= 1e-5, (W, H, kind, w, d, e)
