"""Randomised parity sweep through the C ABI against the oracle (fixed seed, 300 trials):
random frame sizes, windows, strides, levels, supports (row-run and generic kernels), iteration
limits, robust modes (Hampel, L2, hard threshold) and the illumination model, on layered-motion
pairs.  Both sides track the oracle's points and interpolate the oracle's tracks.  Bars:
  * detection: selections exact, points within 1e-3 px (FP32 division against FP64);
  * detection beside the pyramids: points and every pyramid level bit-identical to the separate
    calls;
  * tracking, Hampel and L2 without the illumination model, supports 5 x 5 and larger: every
    point both sides report CONVERGED within 1e-3 px; statuses differ on at most max(1, 0.1 %)
    per trial, and agree on at least 99.9 % of all such points over the sweep;
  * tracking with hard thresholding, the illumination model or a 3 x 3 support: at most
    max(3, 1 %) of the points both sides report CONVERGED lie further apart; statuses differ on
    at most max(3, 2 %) of the points whose coarse levels all stopped on the step test in the
    oracle (determined paths, as in tests/parity.py) and on at most 5 % of all points per trial;
    over the sweep statuses agree on at least 99.9 % of the determined paths (99.8 % for hard
    thresholding with the illumination model) and on at least 99.5 % of all points.  A discontinuous weight, a gain near its acceptance bound trading off
    against the motion, or a nine-pixel system lets FP32 and FP64 iterations settle at different
    fixed points (a 5,000-trial sweep found at most 9 such points in one trial, none with Hampel
    or L2 alone at supports of 5 and up), and a coarse level that runs out of iterations hands on
    an iterate that then depends on rounding (with the illumination model on a 5 x 5 support and
    15 iterations, 15 of 179 such points settled differently, 2 of the 437 others);
  * dense interpolation (frames up to 60,000 pixels): cells and neighbour lists exact.
A second sweep (120 trials) covers the RLOF(IM-GM) options; its bars are at _trial_options."""
import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth

pytestmark = pytest.mark.gpu
RUN = [5, 7, 9, 11, 15, 21]
GEN = [3, 13, 17, 19, 23, 25, 27, 29, 31]
MODES = [dict(sigma1=8.0, sigma2=32.0), dict(sigma1=float("inf"), sigma2=float("inf")),
         dict(sigma1=12.0, sigma2=12.0)]


def _trial(rng, t, tally):
    W, H = int(rng.integers(12, 400)), int(rng.integers(12, 300))
    disp = float(rng.uniform(0, 25))
    I0, I1, _, _ = synth.layered_pair(W, H, seed=int(rng.integers(1 << 30)), max_disp=disp)
    win = int(rng.integers(1, min(W, H, 31) + 1))
    stride = int(rng.integers(1, 13))
    while oracle.detect_count(W, H, win, stride) > 5000:
        stride += 1
    levels, iters = int(rng.integers(1, 7)), int(rng.integers(1, 21))
    illum = bool(rng.random() < 0.25)
    s = int(rng.choice(RUN)) if illum or rng.random() < 0.6 else int(rng.choice(GEN))
    mode = int(rng.integers(3))
    kk = int(rng.choice([1, 8, 64, 128]))
    tag = f"#{t} {W}x{H} w{win} d{stride} L{levels} s{s} it{iters} mode{mode}{' IM' if illum else ''}"
    print(tag, flush=True)
    a, b = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    n = dgf.detect_count(W, H, win, stride)
    P, sel, _ = dgf.detect(a, win, stride, return_sel=True, return_response=True)
    oP, osel, _ = oracle.detect(I0, win, stride)
    if n:
        assert np.array_equal(sel.cpu().numpy(), osel), tag
        assert np.abs(P.cpu().numpy().astype(np.float64) - oP).max() <= 1e-3, tag
    ws1 = torch.zeros(max(dgf.track_workspace_bytes(W, H, levels, 0), 1), dtype=torch.uint8, device="cuda")
    ws2 = torch.ones_like(ws1)
    P2 = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    dgf.track_pyramids(a, b, levels, ws1)
    dgf.detect_pyramids(a, b, win, stride, levels, ws2, P2)
    torch.cuda.synchronize()
    assert torch.equal(P2.view(torch.int32), P.view(torch.int32)), tag
    total, off, pit = dgf.pyramid_layout(W, H, levels, 0)
    Wl, Hl = W, H
    for l in range(1, levels):
        Wl, Hl = (Wl + 1) // 2, (Hl + 1) // 2
        for f in range(2):
            o = f * total + off[l]
            assert torch.equal(ws1[o:o + pit[l] * Hl].view(Hl, pit[l])[:, :Wl],
                               ws2[o:o + pit[l] * Hl].view(Hl, pit[l])[:, :Wl]), (tag, l, f)
    if n == 0:
        return
    # both sides track the oracle's points (FP32, as the tracker takes them)
    Pn = oP.astype(np.float32)
    Pg = torch.from_numpy(Pn).cuda()
    F, S = dgf.track(a, b, Pg, levels, s, iters, opts=dgf.TrackOpts(illum=illum, **MODES[mode]))
    torch.cuda.synchronize()
    gF, gS = F.cpu().numpy().astype(np.float64), S.cpu().numpy()
    oF, oS, oIt = oracle.track(I0, I1, Pn.astype(np.float64), levels, s, iters, illum=illum, return_iters=True,
                               **MODES[mode])[:3]
    both = (gS == 0) & (oS == 0)
    bad = int((np.abs(gF[both] - oF[both]).max(1) > 1e-3).sum()) if both.any() else 0
    differ = int((gS != oS).sum())
    # determined paths: every coarse level stopped on the step test in the oracle
    det = np.all(np.asarray(oIt).reshape(n, -1)[:, :-1] < iters, axis=1)
    differ_det = int(((gS != oS) & det).sum())
    print(f"  n={n} both={int(both.sum())} far={bad} status_differ={differ} "
          f"(determined paths {int(det.sum())}: {differ_det})", flush=True)
    cls = ("illum " if illum else "") + ("hard" if mode == 2 else ("s3" if s == 3 else "smooth"))
    tot = tally.setdefault(cls, [0, 0, 0, 0])
    tot[0] += n
    tot[1] += differ
    tot[2] += int(det.sum())
    tot[3] += differ_det
    if illum or mode == 2 or s == 3:
        assert bad <= max(3, 0.01 * both.sum()), tag
        assert differ_det <= max(3, 0.02 * int(det.sum())), tag
        assert differ <= max(3, 0.05 * n), tag
    else:
        assert bad == 0, tag
        assert differ <= max(1, 0.001 * n), tag
    if W * H <= 60000:
        # interpolation of the oracle's tracking result on both sides
        oF32 = oF.astype(np.float32)
        _, aux = dgf.epic(a, Pg, torch.from_numpy(oF32).cuda(), torch.from_numpy(oS).cuda(),
                          opts=dgf.EpicOpts(k=kk), return_aux=True)
        torch.cuda.synchronize()
        _, o = oracle.epic(I0, Pn.astype(np.float64), oF32.astype(np.float64), oS, k=kk, full=True)
        assert np.array_equal(aux["labels"].cpu().numpy(), o["L"]), tag
        assert np.array_equal(aux["nbr"].cpu().numpy(), o["nb"]), tag


def test_randomised_sweep():
    rng = np.random.default_rng(20190125)
    tally = {}
    for t in range(300):
        _trial(rng, t, tally)
    for cls, (n, differ, n_det, differ_det) in sorted(tally.items()):
        agree = 1.0 - differ / max(n, 1)
        agree_det = 1.0 - differ_det / max(n_det, 1)
        print(f"{cls}: {n} points, statuses agree on {agree:.5f} ({agree_det:.5f} on {n_det} determined paths)",
              flush=True)
        if cls == "smooth":
            assert agree >= 0.999, cls
        else:
            assert agree_det >= (0.998 if cls == "illum hard" else 0.999), cls
            assert agree >= 0.995, cls


def _corner_motion(A, W, H):
    cx, cy = 0.5 * (W - 1), 0.5 * (H - 1)
    P = np.array([[-cx, -cy, 1], [cx, -cy, 1], [-cx, cy, 1], [cx, cy, 1]], np.float64)
    return P @ np.asarray(A, np.float64).reshape(2, 3).T


def _trial_options(rng, t, tally):
    """One random trial of the RLOF(IM-GM) options (cross-based supports, global prior, with or
    without the illumination model) against the oracle, both sides on the oracle's points.  Bars
    on the points whose coarse levels all stopped on the step test in the oracle (tests/parity.py,
    paths="determined": small adaptive supports make a coarse level that runs out of iterations
    hand on a rounding-chaotic iterate): smooth norms without the illumination model, every
    CONVERGED-on-both point within 1e-3 px; otherwise at most max(3, 1 %) further.

    The prior couples every point to one model fitted from the first pass.  Where the two models
    agree (motion at the frame corners within 1e-3 px), statuses differ on at most max(3, 2 %) of
    the points.  A first-pass sample that FP32 and FP64 settle differently (an illumination-model
    point near a runaway gain) moves the fit by hundredths of a pixel, and hard-threshold or
    illumination-model points of the second pass can then settle elsewhere: such a trial must use
    the illumination model, keeps its model within 0.5 px at the corners and its statuses within
    max(3, 5 %); at most 5 of the 120 trials may be of that kind."""
    W, H = int(rng.integers(40, 360)), int(rng.integers(40, 260))
    I0, I1, _, _ = synth.layered_pair(W, H, seed=int(rng.integers(1 << 30)), max_disp=float(rng.uniform(0, 25)))
    stride = int(rng.integers(3, 11))
    levels, iters = int(rng.integers(1, 6)), int(rng.integers(5, 21))
    s = int(rng.choice(RUN))
    cross, gm, illum = bool(rng.random() < 0.6), bool(rng.random() < 0.6), bool(rng.random() < 0.3)
    if not (cross or gm):
        cross = True
    mode = int(rng.integers(3))
    tau = float(rng.choice([10.0, 25.0, 60.0]))
    tag = (f"#{t} {W}x{H} d{stride} L{levels} s{s} it{iters} mode{mode} tau{tau}"
           f"{' cross' if cross else ''}{' gm' if gm else ''}{' IM' if illum else ''}")
    print(tag, flush=True)
    pts = oracle.detect(I0, 9, stride)[0].astype(np.float32)
    if len(pts) == 0:
        return
    a, b = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    opts = dgf.TrackOpts(illum=illum, cross=cross, global_motion=gm, cross_tau=tau, **MODES[mode])
    out = dgf.track(a, b, torch.from_numpy(pts).cuda(), levels, s, iters, opts=opts, return_iters=True,
                    return_gm=gm)
    torch.cuda.synchronize()
    gF, gS = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy()
    o = oracle.track(I0, I1, pts.astype(np.float64), levels, s, iters, illum=illum, cross=cross, tau=tau, gm=gm,
                     return_iters=True, return_gm=gm, **MODES[mode])
    oF, oS, oits = o[:3]
    det = np.all(oits[:, :-1] < iters, axis=1)
    both = (gS == 0) & (oS == 0) & det
    bad = int((np.abs(gF[both] - oF[both]).max(1) > 1e-3).sum()) if both.any() else 0
    nd = int(det.sum())
    differ = int(((gS != oS) & det).sum())
    moved = 0.0
    if gm:
        moved = float(np.abs(_corner_motion(out[3].cpu().numpy(), W, H) - _corner_motion(o[3], W, H)).max())
    print(f"  n={len(gS)} determined={nd} both={int(both.sum())} far={bad} status_differ={differ} "
          f"model_corner_diff={moved:.1e}", flush=True)
    tot = tally.setdefault("options", [0, 0, 0])
    tot[0] += nd
    tot[1] += differ
    if illum or mode == 2:
        assert bad <= max(3, 0.01 * both.sum()), tag
    else:
        assert bad == 0, tag
    if moved > 1e-3:
        tot[2] += 1
        assert illum and moved <= 0.5, tag
        assert differ <= max(3, 0.05 * nd), tag
    else:
        assert differ <= max(3, 0.02 * nd), tag


def test_randomised_sweep_rlof_options():
    rng = np.random.default_rng(19010997)
    tally = {}
    for t in range(120):
        _trial_options(rng, t, tally)
    n, differ, moved = tally["options"]
    agree = 1.0 - differ / max(n, 1)
    print(f"options: {n} points on determined paths, statuses agree on {agree:.5f}; "
          f"{moved} trials with a moved prior", flush=True)
    assert agree >= 0.998
    assert moved <= 5
