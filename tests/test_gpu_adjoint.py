"""GPU parity of the implicit adjoint d(flow)/d(I0, I1) (HIP kernel through the C ABI) against
the FP64 oracle gradient, which the CPU suite pins to central finite differences.

Loss: L = sum over points CONVERGED in the forward pass of |u_k - u_gt|^2, points fixed.  Both
adjoints take the oracle's forward result (flow, statuses, dflow) as their input.
Bar: relative L2 error <= 1e-4 on dI0 and on dI1 separately."""
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


def _check_against_oracle(I0, I1, pts, gt, levels, support, iters, opts, min_conv=0.9):
    """Both adjoints at the oracle's forward result: the FP64 tracker converged to 1e-12 gives the
    flow (rounded to FP32, the type the kernel takes) and the statuses, and dflow follows from
    that flow (the forward kernels are held to the oracle in the tracking tests).  Returns the
    oracle's statuses and the GPU gradients."""
    I0d, I1d = I0.astype(np.float64), I1.astype(np.float64)
    P32 = pts.astype(np.float32)
    P = P32.astype(np.float64)
    oflow, ost = oracle.track(I0d, I1d, P, levels, support, iters, sigma1=opts.sigma1, sigma2=opts.sigma2,
                              min_eig=opts.min_eig, eps_fine=1e-12)
    conv = ost == 0
    assert conv.mean() > min_conv
    fl32 = np.where(conv[:, None], oflow, 0.0).astype(np.float32)
    df32 = np.where(conv[:, None], 2.0 * (fl32.astype(np.float64) - gt), 0.0).astype(np.float32)
    t0 = torch.from_numpy(np.ascontiguousarray(I0, np.float32)).cuda()
    t1 = torch.from_numpy(np.ascontiguousarray(I1, np.float32)).cuda()
    dI0, dI1 = torch.zeros_like(t0), torch.zeros_like(t1)
    dgf.track_backward(t0, t1, torch.from_numpy(P32).cuda(), support, torch.from_numpy(fl32).cuda(),
                       torch.from_numpy(ost).cuda(), torch.from_numpy(df32).cuda(), dI0, dI1, opts=opts)
    torch.cuda.synchronize()
    o0, o1 = oracle.track_grad(I0d, I1d, P, support, fl32.astype(np.float64), ost, df32.astype(np.float64),
                               sigma1=opts.sigma1, sigma2=opts.sigma2)
    dI0, dI1 = dI0.cpu().numpy().astype(np.float64), dI1.cpu().numpy().astype(np.float64)
    e0, e1 = _rel(dI0, o0), _rel(dI1, o1)
    print(f"converged={int(conv.sum())}/{len(ost)} rel(dI0)={e0:.2e} rel(dI1)={e1:.2e}", flush=True)
    assert e0 <= REL and e1 <= REL
    return ost, dI0, dI1


def test_crop_128x64_200_points_vs_oracle():
    # the CPU suite checks the oracle gradient pixel by pixel against central finite differences
    # on this same crop
    I0, I1, gt = synth.translation_f32_1242x375()
    I0 = np.ascontiguousarray(I0[:64, :128])
    I1 = np.ascontiguousarray(I1[:64, :128])
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0]
    assert len(pts) == 200
    _check_against_oracle(I0, I1, pts, gt, 3, 9, 100, dgf.TrackOpts(eps_fine=1e-6))


def test_full_1242x375_and_random_direction_fd():
    I0, I1, gt = synth.translation_f32_1242x375()
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 8)[0]
    assert len(pts) == 7130
    opts = dgf.TrackOpts(eps_fine=1e-6)
    ost, dI0, dI1 = _check_against_oracle(I0, I1, pts, gt, 3, 9, 100, opts)
    # directional derivative <grad L, v> against FP64 central differences of the oracle forward,
    # over the points the oracle's forward converged
    P = pts.astype(np.float32).astype(np.float64)
    conv = ost == 0
    rng = np.random.default_rng(0)
    v0 = rng.normal(size=I0.shape)
    v1 = rng.normal(size=I1.shape)
    # a 1e-3 step moves some of the ~577k support residuals across a robust-norm band edge (a
    # kink of the loss) and costs the central difference ~1e-3 of accuracy; with the FP64 forward
    # converged to 1e-12, h = 1e-4 is both smooth enough and far above round-off
    h = 1e-4

    def loss(a, b):
        f, s_ = oracle.track(a, b, P[conv], 3, 9, 100, eps_fine=1e-12)
        assert np.all(s_ == 0)
        e = f - gt
        return float((e * e).sum())

    I0d, I1d = I0.astype(np.float64), I1.astype(np.float64)
    fd = (loss(I0d + h * v0, I1d + h * v1) - loss(I0d - h * v0, I1d - h * v1)) / (2 * h)
    an = float((dI0 * v0).sum() + (dI1 * v1).sum())
    print(f"directional: fd={fd:.6e} gpu={an:.6e} rel={abs(fd - an) / abs(fd):.2e}", flush=True)
    assert abs(fd - an) <= REL * abs(fd)


def test_robust_layered_scene():
    I0, I1, _, _ = synth.layered_pair(400, 240, seed=5, max_disp=30.0, dtype="f32")
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0]
    gt = np.zeros(2)
    # occlusions and 50 iterations: about half the points reach the 1e-12 step test
    _check_against_oracle(I0, I1, pts, gt, 3, 11, 50, dgf.TrackOpts(eps_fine=1e-6), min_conv=0.5)


def test_least_squares_limit():
    I0, I1, gt = synth.noise_translation_pair(160, 96, seed=9, shift=(1.4, 0.6), dtype="f32")
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 7)[0]
    inf = float("inf")
    _check_against_oracle(I0, I1, pts, gt, 3, 9, 100, dgf.TrackOpts(sigma1=inf, sigma2=inf, min_eig=0.0, eps_fine=1e-6))


def test_autograd_function_matches_direct_call():
    I0, I1, gt = synth.noise_translation_pair(128, 96, seed=10, dtype="f32")
    t0 = torch.from_numpy(I0).cuda().requires_grad_(True)
    t1 = torch.from_numpy(I1).cuda().requires_grad_(True)
    pts = torch.from_numpy(oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 8)[0].astype(np.float32)).cuda()
    flow, st = dgf.TrackFn.apply(t0, t1, pts, 3, 9, 30, None)
    conv = (st == 0).float().unsqueeze(1)
    g = torch.tensor(gt, dtype=torch.float32, device="cuda")
    loss = (((flow - g) ** 2) * conv).sum()
    loss.backward()
    dflow = 2.0 * (flow.detach() - g) * conv
    d0 = torch.zeros_like(t0)
    d1 = torch.zeros_like(t1)
    dgf.track_backward(t0.detach(), t1.detach(), pts, 9, flow.detach(), st, dflow, d0, d1)
    torch.cuda.synchronize()
    assert _rel(t0.grad.cpu().numpy().astype(np.float64), d0.cpu().numpy().astype(np.float64)) < 1e-5
    assert _rel(t1.grad.cpu().numpy().astype(np.float64), d1.cpu().numpy().astype(np.float64)) < 1e-5
    assert float(t1.grad.abs().sum()) > 0


def test_non_converged_points_contribute_nothing():
    I0, I1, gt = synth.noise_translation_pair(96, 64, seed=11, dtype="f32")
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    pts = torch.from_numpy(oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 8)[0].astype(np.float32)).cuda()
    flow, st = dgf.track(t0, t1, pts, 3, 9, 20)
    st1 = torch.ones_like(st)  # nothing converged
    d0, d1 = torch.zeros_like(t0), torch.zeros_like(t1)
    dgf.track_backward(t0, t1, pts, 9, flow, st1, torch.ones_like(flow), d0, d1)
    torch.cuda.synchronize()
    assert float(d0.abs().sum()) == 0.0 and float(d1.abs().sum()) == 0.0
    # u8 frames have no gradient
    with pytest.raises(RuntimeError):
        dgf.track_backward(t0.to(torch.uint8), t1.to(torch.uint8), pts, 9, flow, st, flow, d0, d1)


def test_least_squares_fallback_regime():
    # hard thresholding at sigma 0.5 on a pair with N(0, 20) noise: many points converge in the
    # tracker's least-squares fallback regime, where the gradient differentiates sum r g = 0
    # (the CPU suite pins the oracle there to central differences)
    I0, I1, gt = synth.noise_translation_pair(64, 48, seed=21, dtype="f32")
    I1 = (I1.astype(np.float64) + np.random.default_rng(5).normal(0, 20.0, I1.shape)).astype(np.float32)
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0]
    _check_against_oracle(I0, I1, pts, gt, 3, 9, 100, dgf.TrackOpts(sigma1=0.5, sigma2=0.5, eps_fine=1e-6),
                          min_conv=0.4)
