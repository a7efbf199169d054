"""GPU test of the launch-shape autotuner: it returns a compiled shape, installs it, tracking with
it stays within parity of the oracle, and its JSON cache is written and then hit."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1901_09971_amd as dgf
from paper_1901_09971_amd import synth
from parity import compare_tracks

pytestmark = pytest.mark.gpu


def test_autotune_installs_and_caches(tmp_path):
    before = dgf.get_tuning(21, 4, 0, 0)
    I0, I1, _, _ = synth.layered_pair(480, 256, seed=7, max_disp=50.0)
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    P = oracle.detect(I0, 9, 6)[0].astype(np.float32)
    pts = torch.from_numpy(P).cuda()
    cache = str(tmp_path / "tune.json")
    best = dgf.autotune(t0, t1, pts, 4, 21, 20, cache_path=cache)
    assert best["lanes_per_point"] in (16, 32, 64) and best["ms"] > 0
    cur = dgf.get_tuning(21, 4, 0, pts.shape[0])
    assert all(cur[k] == best[k] for k in ("lanes_per_point", "waves_per_group", "margin", "kernel"))
    with open(cache) as f:
        entries = json.load(f)
    assert len(entries) == 1 and list(entries.values())[0]["lanes_per_point"] == best["lanes_per_point"]
    # a cache hit returns the stored shape (and its stored time) without a new search
    again = dgf.autotune(t0, t1, pts, 4, 21, 20, cache_path=cache)
    assert again == {k: (round(v, 4) if k == "ms" else v) for k, v in best.items()} or \
        all(again[k] == best[k] for k in ("lanes_per_point", "waves_per_group", "margin", "kernel"))
    # tracking with the installed shape is still within parity of the oracle
    flow, st = dgf.track(t0, t1, pts, 4, 21, 20)
    # a cache hit still leaves a tracking result made with the installed shape
    _, hf, hs = dgf.autotune(t0, t1, pts, 4, 21, 20, cache_path=cache, return_result=True)
    torch.cuda.synchronize()
    fin = torch.isfinite(flow)
    assert torch.equal(hs, st) and torch.equal(torch.isfinite(hf), fin) and torch.equal(hf[fin], flow[fin])
    of, ost = oracle.track(I0, I1, P.astype(np.float64), 4, 21, 20)
    compare_tracks(flow.cpu().numpy(), st.cpu().numpy(), of, ost, 0.999, 1e-3, label="autotuned shape")
    dgf.set_tuning(21, 0, before["lanes_per_point"], before["waves_per_group"], before["margin"], before["kernel"])


def test_illumination_model_cached_under_its_own_key(tmp_path):
    before = dgf.get_tuning(21, 4, 0, 0)
    I0, I1, _, _ = synth.layered_pair(320, 200, seed=9, max_disp=20.0)
    t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
    pts = dgf.detect(t0, 9, 8)
    cache = str(tmp_path / "tune.json")
    dgf.autotune(t0, t1, pts, 3, 21, 10, cache_path=cache)
    # the same request with the illumination model is a miss, timed and stored beside the first
    im = dgf.autotune(t0, t1, pts, 3, 21, 10, opts=dgf.TrackOpts(illum=True), cache_path=cache)
    assert im["lanes_per_point"] in (16, 32, 64) and im["ms"] > 0
    with open(cache) as f:
        keys = sorted(json.load(f))
    assert len(keys) == 2 and keys[1] == keys[0] + ":illum", keys
    dgf.set_tuning(21, 0, before["lanes_per_point"], before["waves_per_group"], before["margin"], before["kernel"])
