"""Parity at the density-stress size, in the launch configuration the benchmark times: four
2048x1024 uint8 pairs (layered affine motion up to 250 px, seeds 0-3), DeGraF window 9 stride 2
(518,160 points each), 6 levels, 21x21 support, 20 iterations, one batched plan.  The FP64 oracle
checks every detected point, and the tracking and the adjoint on a seeded sample of points of
every pair (the oracle tracks points one by one)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth
from parity import compare_tracks

pytestmark = pytest.mark.gpu
L, S_, IT, WIN, STRIDE, NPAIRS, SAMPLE = 6, 21, 20, 9, 2, 4, 300


@pytest.fixture(scope="module")
def batch():
    with ThreadPoolExecutor(NPAIRS) as ex:
        data = list(ex.map(synth.density_2048x1024, range(NPAIRS)))
    pairs = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), WIN, STRIDE) for a, b, _, _ in data]
    plan = dgf.Batch(pairs, L, S_, IT)
    P, F, S = plan.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    samples = [rng.choice(plan.offsets[i + 1] - plan.offsets[i], SAMPLE, replace=False) for i in range(NPAIRS)]
    yield data, plan, P, F, S, samples
    plan.close()


def test_every_point_detected(batch):
    data, plan, P, _, _, _ = batch
    Pn = P.cpu().numpy().astype(np.float64)
    for i, (I0, _, _, _) in enumerate(data):
        ref = oracle.detect(I0, WIN, STRIDE)[0]
        lo, hi = plan.offsets[i], plan.offsets[i + 1]
        assert hi - lo == len(ref) == 518160
        assert np.max(np.abs(Pn[lo:hi] - ref)) <= 1e-3


def test_tracking_sample(batch):
    data, plan, P, F, S, samples = batch
    Pn, Fn, Sn = P.cpu().numpy(), F.cpu().numpy().astype(np.float64), S.cpu().numpy()
    g_all, o_all = [], []
    for i, (I0, I1, _, _) in enumerate(data):
        idx = plan.offsets[i] + samples[i]
        pts = Pn[idx].astype(np.float64)
        of, os_ = oracle.track(I0, I1, pts, L, S_, IT)
        r = compare_tracks(Fn[idx], Sn[idx], of, os_, 0.99, 1e-3, label=f"pair {i}")
        assert r["conv"] >= 0.2 * SAMPLE
        g_all.append(Sn[idx])
        o_all.append(os_)
    # over the whole sample (1,200 points) at most one status may differ
    agree = float(np.mean(np.concatenate(g_all) == np.concatenate(o_all)))
    print(f"status agreement over the sample {agree:.5f}", flush=True)
    assert agree >= 0.999


def test_adjoint_sample(batch):
    data, plan, P, F, S, samples = batch
    Sn = S.cpu().numpy()
    g = np.random.default_rng(1)
    dflow = torch.zeros_like(F)
    for i in range(NPAIRS):
        idx = plan.offsets[i] + samples[i]
        idx = idx[Sn[idx] == 0]
        dflow[torch.from_numpy(idx).cuda()] = torch.from_numpy(g.normal(size=(len(idx), 2)).astype(np.float32)).cuda()
    _, views = plan.backward(dflow)
    torch.cuda.synchronize()
    Pn, Fn, Dn = P.cpu().numpy(), F.cpu().numpy(), dflow.cpu().numpy()
    for i, (I0, I1, _, _) in enumerate(data):
        idx = plan.offsets[i] + samples[i]
        o0, o1 = oracle.track_grad(I0.astype(np.float64), I1.astype(np.float64), Pn[idx].astype(np.float64), S_,
                                   Fn[idx].astype(np.float64), Sn[idx], Dn[idx].astype(np.float64))
        for got, ref in ((views[i][0], o0), (views[i][1], o1)):
            got = got.cpu().numpy().astype(np.float64)
            rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print(f"pair {i}: adjoint rel-L2 {rel:.2e}", flush=True)
            assert rel <= 1e-4
