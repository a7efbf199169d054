"""GPU parity of the rest of the RLOF(IM-GM) configuration (Section 3 "Parameters") against the
FP64 oracle, through the C ABI: adaptive cross-based supports (DGF_TRACK_CROSS), the global-motion
prior (DGF_TRACK_GLOBAL) and both with the illumination model.

Bars: as for the plain tracker, flow within 1e-3 px on points converged on both sides and statuses
equal on >= 99.9 % of the points -- on the driving pair for every point, on the small layered
scenes (small supports along many layer borders) for the points whose coarse levels all stopped on
the step test (tests/parity.py, paths="determined"; >= 99 % agreement over all points).  The robust global fit (dgf_gm_fit) on identical samples: every
model coefficient within 1e-9 of the oracle's, relative to the motion it predicts at the frame
corners.  Inside the tracker the fit sees the GPU's own FP32 first pass, so there the two models
are compared by the motion they predict at the frame corners, within 0.05 px.  A batch plan with
the prior must reproduce per-pair calls bit for bit (each pair's fit is reduced the same way)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth
from paper_1901_09971_amd._lib import DgfError
from parity import compare_tracks

pytestmark = pytest.mark.gpu
TOL = 1e-3


def _illum_u8(I1, gain, offset):
    return np.clip(np.rint(gain * I1.astype(np.float64) + offset), 0, 255).astype(np.uint8)


def _run(I0, I1, pts32, L, s, iters, min_agree=0.999, illum=False, cross=False, gm=False, label="", paths="all",
         ill_tol=None):
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    P = torch.from_numpy(pts32).cuda()
    opts = dgf.TrackOpts(illum=illum, cross=cross, global_motion=gm)
    out = dgf.track(t0, t1, P, L, s, iters, opts=opts, return_iters=True, return_gm=gm)
    torch.cuda.synchronize()
    g_flow, g_st, g_its = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy(), out[2].cpu().numpy()
    o = oracle.track(I0, I1, pts32.astype(np.float64), L, s, iters, illum=illum, cross=cross, gm=gm,
                     return_iters=True, return_gm=gm)
    o_flow, o_st, o_its = o[0], o[1], o[2]
    print(f"{label}: {len(pts32)} points", flush=True)
    compare_tracks(g_flow, g_st, o_flow, o_st, min_agree, TOL, g_its=g_its, o_its=o_its, iters=iters, label=label,
                   paths=paths, ill_tol=ill_tol)
    if gm:
        _same_motion(out[3].cpu().numpy(), o[3], I0.shape[1], I0.shape[0], 0.05, label)
    return g_flow, g_st, o_flow, o_st


def _corner_motion(A, W, H):
    cx, cy = 0.5 * (W - 1), 0.5 * (H - 1)
    P = np.array([[-cx, -cy, 1], [cx, -cy, 1], [-cx, cy, 1], [cx, cy, 1]], np.float64)
    return P @ np.asarray(A, np.float64).reshape(2, 3).T


def _same_motion(A_gpu, A_orc, W, H, tol, label=""):
    d = np.abs(_corner_motion(A_gpu, W, H) - _corner_motion(A_orc, W, H)).max()
    print(f"{label}: model gpu {np.round(np.asarray(A_gpu).ravel(), 6)} oracle {np.round(np.asarray(A_orc).ravel(), 6)}"
          f" corner diff {d:.2e}", flush=True)
    assert d <= tol, (label, d)


# ---- cross-based supports


def test_cross_driving_1242x375():
    I0, I1, _, _ = synth.driving_1242x375()
    pts = oracle.detect(I0, 9, 5)[0].astype(np.float32)
    _run(I0, I1, pts, 5, 21, 20, cross=True, label="cross driving")


@pytest.mark.parametrize("s", [5, 7, 9, 11, 15, 21])
def test_cross_supports(s):
    I0, I1, _, _ = synth.layered_pair(320, 240, seed=4, max_disp=30.0)
    pts = oracle.detect(I0, 9, 6)[0].astype(np.float32)
    _run(I0, I1, pts, 4, s, 20, cross=True, label=f"cross s{s}", paths="determined")


@pytest.mark.parametrize("s,tune", [(21, "16,2,2,0"), (21, "32,1,3,0"), (21, "64,4,2,0"), (15, "16,1,2,0"),
                                    (9, "16,4,3,0")])
def test_cross_launch_shapes(s, tune, monkeypatch):
    monkeypatch.setenv("DGF_TUNE", tune)
    I0, I1, _, _ = synth.layered_pair(320, 240, seed=5, max_disp=30.0)
    pts = oracle.detect(I0, 9, 7)[0].astype(np.float32)
    _run(I0, I1, pts, 4, s, 20, cross=True, label=f"cross s{s} {tune}", paths="determined")


def test_cross_float_frames_and_tau():
    I0, I1, _, _ = synth.layered_pair(256, 192, seed=6, max_disp=20.0, dtype="f32")
    pts = oracle.detect(np.clip(np.rint(I0), 0, 255).astype(np.uint8), 9, 6)[0].astype(np.float32)
    _run(I0, I1, pts, 3, 15, 20, cross=True, label="cross f32", paths="determined")
    # tau = 0 keeps only runs of exactly equal pixel values (near nothing on these frames), and a
    # huge tau is the whole square window (the region is the extended patch, so the erosion by the
    # gradient stencil removes nothing)
    t0, t1, P = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), torch.from_numpy(pts).cuda()
    for tau in (0.0, 1e6):
        f, st, its = dgf.track(t0, t1, P, 3, 15, 20, opts=dgf.TrackOpts(cross=True, cross_tau=tau), return_iters=True)
        of, ost, oits = oracle.track(I0, I1, pts.astype(np.float64), 3, 15, 20, cross=True, tau=tau,
                                     return_iters=True)
        compare_tracks(f.cpu().numpy(), st.cpu().numpy(), of, ost, 0.999, TOL, g_its=its.cpu().numpy(), o_its=oits,
                       iters=20, label=f"cross tau={tau}", paths="determined")


def test_cross_with_illumination():
    I0, I1, _, _ = synth.layered_pair(320, 240, seed=7, max_disp=30.0)
    I1 = _illum_u8(I1, 1.1, -6.0)
    pts = oracle.detect(I0, 9, 6)[0].astype(np.float32)
    _run(I0, I1, pts, 4, 21, 20, illum=True, cross=True, label="cross+illum", paths="determined", ill_tol=1e-2)


# ---- global-motion prior


def _samples(n, W, H, seed, outliers=0.2, bad=0.1):
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.uniform(0, W - 1, n), rng.uniform(0, H - 1, n)], 1).astype(np.float32)
    A = np.array([[0.02, -0.01, 12.5], [0.005, 0.03, -4.0]])
    x = np.c_[pts.astype(np.float64) - [0.5 * (W - 1), 0.5 * (H - 1)], np.ones(n)]
    mot = x @ A.T + rng.normal(0, 0.3, (n, 2))
    k = rng.random(n) < outliers
    mot[k] = rng.uniform(-80, 80, (int(k.sum()), 2))
    mot = mot.astype(np.float32)
    st = np.where(rng.random(n) < bad, rng.integers(1, 4, n), 0).astype(np.uint8)
    if n > 10:
        mot[3, 0] = np.nan  # a converged point with a non-finite flow is no sample
        mot[5, 1] = np.inf
    return pts, mot, st


def _fit_both(pts, mot, st, W, H, scale):
    g = dgf.gm_fit(torch.from_numpy(pts).cuda(), torch.from_numpy(mot).cuda(), torch.from_numpy(st).cuda(), W, H,
                   scale).cpu().numpy()
    use = (st == 0) & np.all(np.isfinite(mot), 1)
    o, kind = oracle.gm_fit(pts.astype(np.float64), mot.astype(np.float64), use.astype(np.uint8),
                            (0.5 * (W - 1), 0.5 * (H - 1)), scale)
    return g, np.asarray(o).reshape(2, 3), kind


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 2047, 2048, 2049, 50000, 600000])
def test_gm_fit_matches_oracle(n):
    W, H = 1242, 375
    pts, mot, st = _samples(n, W, H, seed=n)
    g, o, kind = _fit_both(pts, mot, st, W, H, 2.0)
    scale = 1.0 + np.abs(_corner_motion(o, W, H)).max()
    err = np.abs(_corner_motion(g, W, H) - _corner_motion(o, W, H)).max() / scale
    print(f"n={n} kind={kind} gpu={g.ravel()} oracle={o.ravel()} rel={err:.2e}", flush=True)
    assert err <= 1e-9
    if n >= 2048:
        assert kind == 2 and np.abs(g - [[0.02, -0.01, 12.5], [0.005, 0.03, -4.0]]).max() < 0.05


def test_gm_fit_degenerate_cases():
    W, H = 640, 480
    # collinear positions: the weighted mean motion
    pts = np.stack([np.linspace(10, 600, 50), np.full(50, 100.0)], 1).astype(np.float32)
    mot = np.tile([[3.0, -2.0]], (50, 1)).astype(np.float32)
    st = np.zeros(50, np.uint8)
    g, o, kind = _fit_both(pts, mot, st, W, H, 8.0)
    assert kind == 1 and np.allclose(g, [[0, 0, 3.0], [0, 0, -2.0]], atol=1e-12) and np.allclose(g, o, atol=1e-12)
    # no converged point: the zero model
    g, o, kind = _fit_both(pts, mot, np.full(50, 1, np.uint8), W, H, 8.0)
    assert kind == 0 and not g.any() and not o.any()
    # bad arguments are rejected before any launch
    T = torch.zeros((4, 2), device="cuda")
    S = torch.zeros(4, dtype=torch.uint8, device="cuda")
    for kw in (dict(width=0, height=5, scale=1.0), dict(width=5, height=5, scale=0.0),
               dict(width=5, height=5, scale=float("nan"))):
        with pytest.raises(DgfError):
            dgf.gm_fit(T, T, S, **kw)


def test_gm_layered_640x480():
    I0, I1, _, _ = synth.layered_pair(640, 480, seed=8, max_disp=60.0)
    pts = oracle.detect(I0, 9, 6)[0].astype(np.float32)
    _run(I0, I1, pts, 4, 21, 20, gm=True, label="gm layered")


def test_gm_single_level_and_small_support():
    I0, I1, _ = synth.translation_256x128()
    pts = oracle.detect(I0, 9, 8)[0].astype(np.float32)
    _run(I0, I1, pts, 1, 9, 20, gm=True, label="gm L1")
    _run(I0, I1, pts, 3, 7, 10, gm=True, label="gm L3 s7")


def test_im_gm_driving_1242x375():
    """All of RLOF(IM-GM): illumination model, cross-based supports and the global prior.  The
    guesses of ill-conditioned points are held to eps_coarse (1e-2 px): with the 4 x 4 systems on
    small supports some coarse levels converge slowly, and the oracle alone, on points moved by
    1e-5 px, already moves such a guess by 4.6e-3 px."""
    I0, I1, _, _ = synth.driving_1242x375()
    I1 = _illum_u8(I1, 1.08, -7.0)
    pts = oracle.detect(I0, 9, 5)[0].astype(np.float32)
    _run(I0, I1, pts, 5, 21, 20, illum=True, cross=True, gm=True, label="IM-GM driving", paths="determined",
         ill_tol=1e-2)


@pytest.mark.parametrize("flags", [dict(global_motion=True), dict(global_motion=True, cross=True, illum=True)])
def test_gm_batch_equals_per_pair(flags):
    sizes = [(1242, 375), (640, 480), (320, 240), (77, 41)]
    strides = [5, 8, 3, 4]
    pairs = []
    for i, (W, H) in enumerate(sizes):
        I0, I1, _, _ = synth.layered_pair(W, H, seed=200 + i, max_disp=60.0 * W / 1242.0)
        pairs.append((torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), 9, strides[i]))
    opts = dgf.TrackOpts(**flags)
    plan = dgf.Batch(pairs, 4, 21, 20, opts=opts)
    P, F, S = [t.clone() for t in plan.run()]
    pts, flow, st = [], [], []
    for a, b, w, d in pairs:
        p = dgf.detect(a, w, d)
        f, s = dgf.track(a, b, p, 4, 21, 20, opts=opts)
        pts.append(p)
        flow.append(f)
        st.append(s)
    p, f, s = torch.cat(pts), torch.cat(flow), torch.cat(st)
    torch.cuda.synchronize()
    assert torch.equal(P, p) and torch.equal(S, s)
    fin = torch.isfinite(f)
    assert torch.equal(torch.isfinite(F), fin) and torch.equal(F[fin], f[fin])
    # and a graph replay of the plan reproduces its eager run (the fit's launches included)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.capture()
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(side):
            plan.flow.zero_()
            plan.status.fill_(255)
            plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(plan.status, S), rep
        assert torch.equal(plan.flow[fin], F[fin]), rep
        torch.randn(1 << 18, device="cuda").sum().item()  # eager work between replays
    plan.close()


def test_gm_adjoint_accepts_the_prior_and_cross_is_rejected():
    I0, I1, _ = synth.noise_translation_pair(96, 64, seed=2, shift=(1.3, -0.8), dtype="f32")
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    pts = torch.tensor([[40.0, 30.0], [50.5, 20.25]], device="cuda")
    f, st = dgf.track(t0, t1, pts, 2, 9, 20, opts=dgf.TrackOpts(global_motion=True))
    df = torch.ones_like(f)
    g = [torch.zeros_like(t0), torch.zeros_like(t1)]
    h = [torch.zeros_like(t0), torch.zeros_like(t1)]
    dgf.track_backward(t0, t1, pts, 9, f, st, df, g[0], g[1], opts=dgf.TrackOpts(global_motion=True))
    dgf.track_backward(t0, t1, pts, 9, f, st, df, h[0], h[1])
    torch.cuda.synchronize()
    assert torch.equal(g[0], h[0]) and torch.equal(g[1], h[1])
    with pytest.raises(DgfError):
        dgf.track_backward(t0, t1, pts, 9, f, st, df, g[0], g[1], opts=dgf.TrackOpts(cross=True))
