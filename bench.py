#!/usr/bin/env python3
"""Throughput of the DeGraF detection + robust pyramidal tracking hot path on one MI355X.

One step = DeGraF key-point detection on I0, the pyramids of both frames, and robust tracking of
every detected point, on one 1242x375 driving-shaped uint8 pair (window 9, stride 5: 18,278
points; 5 pyramid levels, 21x21 support, at most 20 iterations per level).  The frames are
resident in device memory before the timed region; every step recomputes everything, in two
launches: detection beside both pyramids (dgf_detect_pyramids), then tracking
(``--separate-detect``: detection, pyramids and tracking as three launches).

Prints ONE JSON line.  ``value`` is tracked points per second over the timed steps.  The
``roofline`` object describes the dominant kernel (the tracker): its algorithmic FP32 work per
launch (24 flops per executed support-pixel iteration, counted from the per-point iteration
numbers the kernel reports) over its average duration measured with HIP events on the stream it
runs on.  ``achievable`` holds the on-box peak probes; ``kernels`` gives every kernel of every
workload (the small translation pair, the benchmark pair, the 64-pair batch, the density stress)
its roofline time from algorithmic counts against the nominal and the achievable peak, and each
workload a sum-of-rooflines over measured time.  ``cpu_baseline`` times the FP64 CPU oracle on
the host cores: the benchmark pair, and bounded samples of the other workloads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tracked points/sec (DeGraF+RLOF) @1242x375; batched vs plain frame-pairs/sec"
FLOPS_PER_PIXEL_ITER = 24          # per support pixel per iteration: bilinear 7, residual 1, weight 3, psi 1, sums 12
PEAK_FP32_VALU_TFLOPS = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, unpacked FP32
PEAK_HBM_GBPS = 8000.0
PEAK_LANE_INSTR = 39.3e12          # unpacked FP32 VALU issue: 256 CU x 64 lanes x 2.4 GHz
INSTR_PER_PIXEL_ITER = 16          # algorithmic lane-instructions per pixel-iteration: bilinear 4 FMA (residual
                                   # folded in), robust weight 4, w*g 2 mul, five accumulations 5 FMA, +1 slack
C1 = dict(name="translation_256x128", W=256, H=128, window=9, stride=8, levels=3, support=9, iters=10)
WORKLOAD = dict(name="driving_1242x375", W=1242, H=375, window=9, stride=5, levels=5, support=21, iters=20)
COUNTERS_FILE = os.path.join(ROOT, "profiles", "track_driving_1242x375_counters.md")
TRACK_SOURCES = ["paper_1901_09971_amd/csrc/track.hip", "paper_1901_09971_amd/csrc/track_kernel.hpp",
                 "paper_1901_09971_amd/csrc/track_run_kernel.hpp", "paper_1901_09971_amd/csrc/dgf_internal.hpp"]


def track_source_sha() -> str:
    h = hashlib.sha256()
    for rel in TRACK_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic():
    """HBM bytes per track launch from the committed rocprofv3 counter summary, or None when
    the summary is missing or was taken on a different version of the kernel source."""
    try:
        with open(COUNTERS_FILE) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"<!--\s*machine:\s*(\{.*?\})\s*-->", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha") != track_source_sha():
        return None
    return d


def cpu_baseline(I0, I1, n_points, budget_s, interp=False):
    import numpy as np

    import oracle  # the CPU baseline leg is the only product-side user of the oracle
    w = WORKLOAD
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores)
    t0 = time.perf_counter()
    reps = 0
    while True:
        pts, _, _ = oracle.detect(I0, w["window"], w["stride"], threads=threads)
        flow, st = oracle.track(I0, I1, pts, w["levels"], w["support"], w["iters"], threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 100:
            break
    # one thread on a bounded sample of the same pair (every 8th point)
    sub = np.ascontiguousarray(pts[::8])
    t1 = time.perf_counter()
    oracle.track(I0, I1, sub, w["levels"], w["support"], w["iters"], threads=1)
    el1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    res = {"value": reps * n_points / el, "unit": "points/s", "cores": threads, "kind": "oracle",
           "sample": f"{reps} full pass(es) of detect+track of the {n_points}-point 1242x375 pair, FP64, "
                     f"{el:.1f} s wall",
           "single_thread_value": len(sub) / el1,
           "single_thread_sample": f"track of every 8th point ({len(sub)}), 1 thread, {el1:.1f} s",
           "cpu_model": model}
    if interp:
        # the dense interpolation of the oracle's own tracks of the same pair (geodesic partition
        # single-threaded, neighbour searches and fits over the host threads)
        t2 = time.perf_counter()
        oracle.epic(I0, pts, flow, st)
        res["interpolation_s"] = time.perf_counter() - t2
    return res


def batched_vs_plain(reps: int, peaks: dict | None = None):
    """Frame-pairs/s on the 64-pair mixed set (four sizes, strides 3/5/8; 5 levels, 21x21, 20
    iterations): per-pair launches (detect, 4 pyramid levels, track for each pair in turn) vs one
    replay of the captured batched plan.  Same tracker launch shape in both.  The plan's two
    halves (pyramids + detection, tracking) are also timed on their own for their rooflines."""
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    L_, s_, it_ = 5, 21, 20
    data = synth.batch64_mixed()
    dev = torch.device("cuda", 0)
    pairs = [(torch.from_numpy(d["I0"]).to(dev), torch.from_numpy(d["I1"]).to(dev), 9, d["stride"]) for d in data]
    # plain: preallocated per-pair buffers
    bufs = []
    for a, b, w, d in pairs:
        n = dgf.detect_count(a.shape[1], a.shape[0], w, d)
        bufs.append(dict(p=torch.empty((n, 2), dtype=torch.float32, device=dev),
                         f=torch.empty((n, 2), dtype=torch.float32, device=dev),
                         s=torch.empty(n, dtype=torch.uint8, device=dev),
                         ws=torch.empty(dgf.track_workspace_bytes(a.shape[1], a.shape[0], L_, 0), dtype=torch.uint8,
                                        device=dev)))

    def plain():
        for (a, b, w, d), B in zip(pairs, bufs):
            dgf.detect(a, w, d, out=B["p"])
            dgf.track_pyramids(a, b, L_, B["ws"])
            dgf.track_run(a, b, B["p"], L_, s_, it_, B["ws"], B["f"], B["s"])

    plan = dgf.Batch(pairs, L_, s_, it_)
    its = torch.empty(plan.num_points, dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan.run(its)
        plan.capture()
    torch.cuda.synchronize()
    pix_iters = int(its.to(torch.int64).sum().item()) * s_ ** 2

    def timed(fn, stream):
        with torch.cuda.stream(stream):
            for _ in range(2):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_plain = timed(plain, side)
    t_batch = timed(plan.replay, side)
    t_front = timed(plan.front, side)
    t_track = timed(plan.track, side)
    # the two forms must agree exactly
    P = torch.cat([B["p"] for B in bufs])
    S = torch.cat([B["s"] for B in bufs])
    identical = bool(torch.equal(P, plan.points) and torch.equal(S, plan.status))
    npts = plan.num_points
    plan.close()
    fb = sum(front_bytes(a.shape[1], a.shape[0], L_, B["p"].shape[0]) for (a, _, _, _), B in zip(pairs, bufs))
    kern = {"front": roof("hbm", fb, t_front, peaks),
            "track": roof("alu", pix_iters * FLOPS_PER_PIXEL_ITER, t_track, peaks, pix_iters)}
    kern["front"]["kernels"] = "k_front_batched (level 1 of every frame beside every pair's detection), k_pyr_level_batched x 3"
    kern["track"]["kernel"] = "k_track_run<64,1,7,31,21,u8,IM=0,HAMPEL,CROSS=0,BATCH=1> (persistent)"
    return {"pairs": len(pairs), "points": npts, "reps": reps,
            "plain_ms": t_plain, "batched_ms": t_batch,
            "plain_pairs_per_s": len(pairs) / (t_plain * 1e-3),
            "batched_pairs_per_s": len(pairs) / (t_batch * 1e-3),
            "speedup": t_plain / t_batch, "identical_outputs": identical,
            "batched_track_tflops_lower_bound": pix_iters * FLOPS_PER_PIXEL_ITER / (t_batch * 1e-3) / 1e12,
            "kernels": kern, "sigma_roofline": sigma_roofline(kern, t_batch),
            "workload": "batch64_mixed: 16 each of 1242x375, 1224x370, 640x480, 320x240, strides {3,5,8}"}


FLOPS_PER_PIXEL_ITER_ILLUM = 39    # illumination model: bilinear 7, residual 2, weight 3, w*(gx, gy, T') 3,
                                   # the ten sums of the 4x4 matrix 16, the four right-hand sums 8


def illumination(steps: int, warmup: int):
    """The benchmark pair with the illumination model (DGF_TRACK_ILLUM) and I1 changed by a gain of
    1.15 and an offset of -12 (rounded to uint8): detection with the pyramids, then tracking, HIP
    events."""
    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    w = WORKLOAD
    I0n, I1n, _, _ = synth.driving_1242x375()
    I1n = np.clip(np.rint(1.15 * I1n.astype(np.float64) - 12.0), 0, 255).astype(np.uint8)
    dev = torch.device("cuda", 0)
    I0, I1 = torch.from_numpy(I0n).to(dev), torch.from_numpy(I1n).to(dev)
    N = dgf.detect_count(w["W"], w["H"], w["window"], w["stride"])
    pts = torch.empty((N, 2), dtype=torch.float32, device=dev)
    flow = torch.empty((N, 2), dtype=torch.float32, device=dev)
    status = torch.empty(N, dtype=torch.uint8, device=dev)
    its = torch.empty(N, dtype=torch.int32, device=dev)
    ws = torch.empty(dgf.track_workspace_bytes(w["W"], w["H"], w["levels"], 0), dtype=torch.uint8, device=dev)
    opts = dgf.TrackOpts(illum=True)
    dgf.detect(I0, w["window"], w["stride"], out=pts)
    dgf.track_pyramids(I0, I1, w["levels"], ws)
    dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, its, opts=opts)
    torch.cuda.synchronize()
    pix_iters = int(its.to(torch.int64).sum().item()) * w["support"] ** 2
    st_counts = np.bincount(status.cpu().numpy(), minlength=4).tolist()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    for _ in range(warmup):
        dgf.detect_pyramids(I0, I1, w["window"], w["stride"], w["levels"], ws, pts)
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, opts=opts)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for e in ev:  # as the main step: front end, then tracking between two events
        dgf.detect_pyramids(I0, I1, w["window"], w["stride"], w["levels"], ws, pts)
        e[0].record()
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, opts=opts)
        e[1].record()
    end.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / steps
    t_track = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    achieved = pix_iters * FLOPS_PER_PIXEL_ITER_ILLUM / (t_track * 1e-3) / 1e12
    return {"workload": "driving_1242x375, I1 gain 1.15 offset -12, illumination model", "points": N,
            "points_per_s": N / (ms_step * 1e-3), "ms_per_step": ms_step, "track_ms": t_track,
            "iterations": pix_iters // w["support"] ** 2, "status_counts": st_counts,
            "flops_per_pixel_iteration": FLOPS_PER_PIXEL_ITER_ILLUM, "achieved_tflops": achieved,
            "frac": achieved / PEAK_FP32_VALU_TFLOPS}


def differentiation(reps: int):
    """The differentiation workload: the 1242x375 FP32 translation pair (shift (2.3, -1.7), 7,130
    points at window 9 stride 8; 3 levels, 9x9 support, 10 iterations), loss = sum over converged
    points of |u - u_gt|^2.  Forward: detect (on the frame rounded to grey levels) + track; backward:
    the tracker adjoint w.r.t. both frames and the points, then the gradient through detection."""
    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    I0n, I1n, gt = synth.translation_f32_1242x375()
    dev = torch.device("cuda", 0)
    I0, I1 = torch.from_numpy(I0n).to(dev), torch.from_numpy(I1n).to(dev)
    u8 = I0.round().clamp(0, 255).to(torch.uint8)
    L_, s_, it_, w_, d_ = 3, 9, 10, 9, 8
    g = torch.tensor(gt, dtype=torch.float32, device=dev)
    pts, sel = dgf.detect(u8, w_, d_, return_sel=True)
    n = pts.shape[0]
    ws = torch.empty(dgf.track_workspace_bytes(1242, 375, L_, 1), dtype=torch.uint8, device=dev)
    flow = torch.empty((n, 2), dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    dI0, dI1 = torch.zeros_like(I0), torch.zeros_like(I1)
    dp = torch.empty_like(pts)
    dflow = torch.zeros_like(flow)

    def fwd():
        dgf.detect(u8, w_, d_, out=pts)
        dgf.track_pyramids(I0, I1, L_, ws)
        dgf.track_run(I0, I1, pts, L_, s_, it_, ws, flow, st)

    def bwd():
        dgf.track_backward(I0, I1, pts, s_, flow, st, dflow, dI0, dI1, dpoints=dp)
        dgf.detect_backward(u8, w_, d_, sel, dp, dI0)

    fwd()
    conv = st == 0
    dflow[conv] = 2.0 * (flow[conv] - g)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_f, t_b = timed(fwd), timed(bwd)
    return {"workload": "translation_f32_1242x375, window 9 stride 8, L3 s9 it10, loss sum |u - u_gt|^2",
            "points": n, "converged": int(conv.sum().item()), "forward_ms": t_f, "backward_ms": t_b,
            "backward_includes": "tracker adjoint w.r.t. I0, I1 and points + gradient through detection"}


def interpolation(reps: int):
    """Dense interpolation (dgf_epic, k = 128) of the benchmark pair's tracked points: the GPU
    detection and tracking output, then the dense field of every pixel.  The call synchronises
    (its geodesic relaxation runs to a fixed point), so it is timed on the host clock; the form
    without host synchronisation (dgf_epic_async) is timed on the stream beside it.  Accuracy:
    endpoint error and > 3 px rate of the dense field on the non-occluded pixels of the synthetic
    ground truth."""
    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    w = WORKLOAD
    I0n, I1n, gt, occ = synth.driving_1242x375()
    dev = torch.device("cuda", 0)
    I0, I1 = torch.from_numpy(I0n).to(dev), torch.from_numpy(I1n).to(dev)
    pts = dgf.detect(I0, w["window"], w["stride"])
    flow, st = dgf.track(I0, I1, pts, w["levels"], w["support"], w["iters"])
    ws = torch.empty(dgf.epic_workspace_bytes(w["W"], w["H"], pts.shape[0]), dtype=torch.uint8, device=dev)
    dense = dgf.epic(I0, pts, flow, st, workspace=ws)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        dense = dgf.epic(I0, pts, flow, st, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    # the form without host synchronisation (dgf_epic_async), timed on the stream with HIP events
    st_out = torch.empty(1, dtype=torch.int32, device=dev)
    dense2 = torch.empty_like(dense)
    dgf.epic_async(I0, pts, flow, st, workspace=ws, dense=dense2, status_out=st_out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dgf.epic_async(I0, pts, flow, st, workspace=ws, dense=dense2, status_out=st_out)
    e1.record()
    torch.cuda.synchronize()
    async_ms = e0.elapsed_time(e1) / reps
    async_same = int(st_out.item()) == 0 and bool(torch.equal(dense2.view(torch.int32), dense.view(torch.int32)))
    d = dense.cpu().numpy().astype(np.float64)
    valid = ~occ
    err = np.linalg.norm(d - gt, axis=-1)[valid]
    P, F, S = pts.cpu().numpy(), flow.cpu().numpy(), st.cpu().numpy()
    conv = S == 0
    xi = np.clip(np.rint(P[conv, 0]).astype(np.int64), 0, w["W"] - 1)
    yi = np.clip(np.rint(P[conv, 1]).astype(np.int64), 0, w["H"] - 1)
    sparse_err = np.linalg.norm(F[conv] - gt[yi, xi], axis=-1)
    return {"workload": "driving_1242x375 tracked points -> dense field, k 128, kappa 8, half-distance 64",
            "seeds": int(conv.sum()), "pixels": w["W"] * w["H"], "reps": reps, "ms": ms,
            "mpix_per_s": w["W"] * w["H"] / (ms * 1e-3) / 1e6,
            "epe_noc_px": float(err.mean()), "outliers_3px_noc": float((err > 3.0).mean()),
            "seed_epe_px": float(sparse_err.mean()),
            "async_ms": async_ms, "async_identical": async_same,
            "async_what": "dgf_epic_async (32 relaxation launches at most, none read back), HIP events"}


DENSITY = dict(name="density_2048x1024x4", W=2048, H=1024, pairs=4, window=9, stride=2, levels=6, support=21,
               iters=20)


def density_stress(reps: int, peaks: dict | None = None):
    """Density stress: four 2048x1024 uint8 pairs (layered affine motion up to 250 px, seeds 0-3),
    DeGraF window 9 stride 2 (518,160 points each), 6 levels, 21x21 support, 20 iterations.
    Forward: one replay of the captured batched plan (detect, pyramids, track of all four pairs).
    Adjoint: one batched backward launch for the loss sum over converged points of |u - u_gt|^2
    (the upstream gradient is formed outside the timed region)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    c = DENSITY
    with ThreadPoolExecutor(c["pairs"]) as ex:
        data = list(ex.map(synth.density_2048x1024, range(c["pairs"])))
    dev = torch.device("cuda", 0)
    pairs = [(torch.from_numpy(I0).to(dev), torch.from_numpy(I1).to(dev), c["window"], c["stride"])
             for I0, I1, _, _ in data]
    plan = dgf.Batch(pairs, c["levels"], c["support"], c["iters"])
    n = plan.num_points
    its = torch.empty(n, dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        P, F, S = plan.run(its)
        plan.capture()
    torch.cuda.synchronize()
    pix_iters = int(its.to(torch.int64).sum().item()) * c["support"] ** 2
    st_counts = np.bincount(S.cpu().numpy(), minlength=4).tolist()

    # upstream gradient of sum over converged points of |u - u_gt|^2 (gt of the nearest pixel)
    pts = P.cpu().numpy()
    gt_pts = np.zeros((n, 2), np.float32)
    for i, (_, _, gt, _) in enumerate(data):
        lo, hi = plan.offsets[i], plan.offsets[i + 1]
        xi = np.clip(np.rint(pts[lo:hi, 0]).astype(np.int64), 0, c["W"] - 1)
        yi = np.clip(np.rint(pts[lo:hi, 1]).astype(np.int64), 0, c["H"] - 1)
        gt_pts[lo:hi] = gt[yi, xi]
    conv = S == 0
    dflow = torch.zeros_like(F)
    dflow[conv] = 2.0 * (F[conv] - torch.from_numpy(gt_pts).to(dev)[conv])
    total, _ = plan.grad_layout()
    grad = torch.empty(total, dtype=torch.float32, device=dev)

    def timed(fn):
        with torch.cuda.stream(side):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_fwd = timed(plan.replay)
    t_front = timed(plan.front)
    t_track = timed(plan.track)
    t_bwd = timed(lambda: plan.backward(dflow, grad))
    # dense interpolation of the first pair's tracked points (the call synchronises: host clock)
    lo, hi = plan.offsets[0], plan.offsets[1]
    I0p = pairs[0][0]
    e_args = (I0p, P[lo:hi].contiguous(), F[lo:hi].contiguous(), S[lo:hi].contiguous())
    dgf.epic(*e_args)
    torch.cuda.synchronize()
    e_times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        dgf.epic(*e_args)
        torch.cuda.synchronize()
        e_times.append(time.perf_counter() - t0)
    plan.close()
    n_conv = int(conv.sum().item())
    per_pair = n // c["pairs"]
    kern = {"front": roof("hbm", c["pairs"] * front_bytes(c["W"], c["H"], c["levels"], per_pair), t_front, peaks),
            "track": roof("alu", pix_iters * FLOPS_PER_PIXEL_ITER, t_track, peaks, pix_iters)}
    # adjoint: reads both frames and the point data, writes both gradient maps (cleared first)
    adj_bytes = c["pairs"] * (2 * c["W"] * c["H"] + 2 * 2 * 4 * c["W"] * c["H"]) + n * (8 + 8 + 8 + 1)
    kern["front"]["kernels"] = "k_front_batched (level 1 of every frame beside every pair's detection), k_pyr_level_batched x 4"
    adj = roof("hbm", adj_bytes, t_bwd, peaks)
    adj["tap_adds_per_s"] = n_conv * c["support"] ** 2 * 10 / (t_bwd * 1e-3)
    adj["what"] = ("bytes: frames read, both gradient maps cleared and written, points/flow/dflow/status read; "
                   "tap adds: 10 per support pixel per converged point (the scatter)")
    return {"workload": c["name"], "pairs": c["pairs"], "points": n, "levels": c["levels"],
            "kernels": dict(kern, adjoint=adj), "sigma_roofline_forward": sigma_roofline(kern, t_fwd),
            "support": c["support"], "max_iters": c["iters"], "reps": reps, "status_counts": st_counts,
            "forward_ms": t_fwd, "forward_points_per_s": n / (t_fwd * 1e-3),
            "forward_track_tflops_lower_bound": pix_iters * FLOPS_PER_PIXEL_ITER / (t_fwd * 1e-3) / 1e12,
            "adjoint_ms": t_bwd, "adjoint_converged_points": n_conv,
            "adjoint_points_per_s": n_conv / (t_bwd * 1e-3),
            "interpolation_ms_one_pair": float(np.median(e_times)) * 1e3,
            "interpolation_seeds_one_pair": int((S[lo:hi] == 0).sum().item())}


def achievable_peaks():
    """On-box probes of what the chip delivers (libdgf_peaks.so, built beside the package): HBM
    stream copy and stream read over 1 GiB buffers (four times the 256 MB Infinity Cache, so the
    stream comes from HBM), LDS read bandwidth (conflict-free 16-byte reads), and the FP32 issue
    rates of unpacked FMA and of the reciprocal, each over ~5 ms launches, HIP events, best of 5."""
    import ctypes

    import torch

    L = ctypes.CDLL(os.path.join(ROOT, "paper_1901_09971_amd", "probes", "libdgf_peaks.so"))
    dev = torch.device("cuda", 0)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n16 = (1 << 30) // 16
    a = torch.ones(n16 * 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    blocks = cus * 8
    out = torch.empty(max(blocks * 256, cus * 32 * 256), dtype=torch.float32, device=dev)

    def best(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    mem_blocks = cus * 32
    t_copy = best(lambda: L.pk_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_int64(n16), mem_blocks, st))
    t_read = best(lambda: L.pk_read(ctypes.c_void_p(a.data_ptr()), ctypes.c_int64(n16),
                                    ctypes.c_void_p(out.data_ptr()), mem_blocks, st))
    it_lds, it_fma, it_rcp = 6000, 6000, 1500
    t_lds = best(lambda: L.pk_lds(it_lds, ctypes.c_void_p(out.data_ptr()), blocks, st))
    t_fma = best(lambda: L.pk_fma(it_fma, ctypes.c_void_p(out.data_ptr()), blocks, st))
    t_rcp = best(lambda: L.pk_rcp(it_rcp, ctypes.c_void_p(out.data_ptr()), blocks, st))
    threads = blocks * 256
    fma_rate = threads * it_fma * 64 / (t_fma * 1e-3)
    rcp_rate = threads * it_rcp * 64 / (t_rcp * 1e-3)
    del a, b, out
    torch.cuda.empty_cache()
    return {"hbm_copy_gbps": 2 * (1 << 30) / (t_copy * 1e-3) / 1e9,
            "hbm_read_gbps": (1 << 30) / (t_read * 1e-3) / 1e9,
            "lds_read_tbps": threads * it_lds * 8 * 16 / (t_lds * 1e-3) / 1e12,
            "fp32_fma_tflops": 2 * fma_rate / 1e12,
            "rcp_per_fma_rate": rcp_rate / fma_rate,
            "compute_units": cus,
            "what": "1 GiB copy (read + write bytes) and read; LDS conflict-free 16-byte reads; "
                    "unpacked FP32 FMA and v_rcp_f32, 8 independent chains per lane"}


def copy_calibration(mib: int):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * 1024 * 1024
    a = torch.empty(n, dtype=torch.uint8, device="cuda").random_(0, 255)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}))


def front_bytes(W: int, H: int, levels: int, n_points: int) -> int:
    """Algorithmic HBM bytes of detection and both pyramids of one pair (per-kernel counts: the
    detector reads the frame and writes 8 B per point; each pyramid reads every level but the
    coarsest and writes every level but the finest)."""
    pyr = 0
    Wl, Hl = W, H
    for _ in range(levels - 1):
        pyr += Wl * Hl
        Wl, Hl = (Wl + 1) // 2, (Hl + 1) // 2
        pyr += Wl * Hl
    return W * H + 8 * n_points + 2 * pyr


def roof(bound: str, amount: float, ms: float, peaks: dict | None, pixel_iters: int | None = None) -> dict:
    """One kernel against its roof: ``amount`` algorithmic bytes (hbm) or flops (alu) per launch
    over ``ms`` per launch, with the roofline time at the nominal and the achievable peak."""
    if bound == "hbm":
        nominal, achievable = PEAK_HBM_GBPS * 1e9, (peaks["hbm_copy_gbps"] * 1e9 if peaks else None)
        unit = "bytes"
    else:
        nominal, achievable = PEAK_FP32_VALU_TFLOPS * 1e12, (peaks["fp32_fma_tflops"] * 1e12 if peaks else None)
        unit = "flops"
    r = {"bound": bound, "ms": ms, "algorithmic": amount, "unit": unit,
         "roofline_ms_nominal": amount / nominal * 1e3, "frac_nominal": amount / nominal * 1e3 / ms}
    if achievable:
        r["roofline_ms_achievable"] = amount / achievable * 1e3
        r["frac_achievable"] = amount / achievable * 1e3 / ms
    if pixel_iters is not None:
        # instruction-issue form: the algorithmic lane-instructions at the unpacked issue rate
        r["issue_frac_nominal"] = pixel_iters * INSTR_PER_PIXEL_ITER / PEAK_LANE_INSTR * 1e3 / ms
        if peaks:
            r["issue_frac_achievable"] = (pixel_iters * INSTR_PER_PIXEL_ITER / (peaks["fp32_fma_tflops"] * 1e12 / 2)
                                          * 1e3 / ms)
    return r


def sigma_roofline(kernels: dict, total_ms: float) -> dict:
    """Sum over kernels of their roofline times, over the measured total."""
    out = {"measured_ms": total_ms}
    for key in ("nominal", "achievable"):
        vals = [k.get("roofline_ms_" + key) for k in kernels.values()]
        if all(v is not None for v in vals):
            out["sum_roofline_ms_" + key] = sum(vals)
            out["frac_" + key] = sum(vals) / total_ms
    return out


def track_kernel_name(tuning: dict | None, support: int, dtype: str = "u8", illum: bool = False,
                      cross: bool = False, batch: bool = False) -> str:
    """The instantiation that runs for a tuning: row-run k_track_run<lanes, runs per lane, run length,
    tile pitch, support, pixel type, illum, robust norm, cross, batch> or the generic k_track."""
    t = tuning or {}
    lpp = int(t.get("lanes_per_point", 64))
    if int(t.get("kernel", 0)) == 0 and support == 21:
        seg = {64: 1, 32: 2, 16: 4}[lpp]
        return (f"k_track_run<{lpp},{seg},7,31,21,{dtype},IM={int(illum)},HAMPEL,CROSS={int(cross)},"
                f"BATCH={int(batch)}>")
    return f"k_track<{lpp},...,{dtype}>"


def lscpu_info() -> dict:
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return info
    keys = {"Model name": "cpu_model", "CPU(s)": "logical_cpus", "Thread(s) per core": "threads_per_core",
            "Core(s) per socket": "cores_per_socket", "Socket(s)": "sockets"}
    for ln in txt.splitlines():
        k, _, v = ln.partition(":")
        if k.strip() in keys:
            info[keys[k.strip()]] = v.strip()
    return info


def c1_step(steps: int, warmup: int, peaks: dict | None):
    """The small translation pair (256x128, window 9 stride 8: 465 points; 3 levels, 9x9, 10
    iterations): the same two-launch step as the benchmark pair, HIP events."""
    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    c = C1
    I0n, I1n, _ = synth.translation_256x128()
    dev = torch.device("cuda", 0)
    I0, I1 = torch.from_numpy(I0n).to(dev), torch.from_numpy(I1n).to(dev)
    N = dgf.detect_count(c["W"], c["H"], c["window"], c["stride"])
    pts = torch.empty((N, 2), dtype=torch.float32, device=dev)
    flow = torch.empty((N, 2), dtype=torch.float32, device=dev)
    status = torch.empty(N, dtype=torch.uint8, device=dev)
    its = torch.empty(N, dtype=torch.int32, device=dev)
    ws = torch.empty(dgf.track_workspace_bytes(c["W"], c["H"], c["levels"], 0), dtype=torch.uint8, device=dev)

    def front():
        dgf.detect_pyramids(I0, I1, c["window"], c["stride"], c["levels"], ws, pts)

    def track(io=None):
        dgf.track_run(I0, I1, pts, c["levels"], c["support"], c["iters"], ws, flow, status, io)

    front()
    track(its)
    torch.cuda.synchronize()
    pix_iters = int(its.to(torch.int64).sum().item()) * c["support"] ** 2
    for _ in range(warmup):
        front()
        track()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for e in ev:
        front()
        e[0].record()
        track()
        e[1].record()
    end.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(end) / steps
    t_track = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    t_front = (start.elapsed_time(ev[0][0]) + sum(ev[k - 1][1].elapsed_time(ev[k][0]) for k in range(1, steps))) / steps
    kern = {"front": roof("hbm", front_bytes(c["W"], c["H"], c["levels"], N), t_front, peaks),
            "track": roof("alu", pix_iters * FLOPS_PER_PIXEL_ITER, t_track, peaks, pix_iters)}
    return {"workload": c["name"], "points": N, "steps": steps, "ms_per_step": ms_step,
            "points_per_s": N / (ms_step * 1e-3), "status_counts": np.bincount(status.cpu().numpy(),
                                                                                minlength=4).tolist(),
            "kernels": kern, "sigma_roofline": sigma_roofline(kern, ms_step)}


def im_gm(steps: int, warmup: int, plain: dict | None):
    """RLOF(IM-GM) on the benchmark pair (illumination model, cross-based supports, global prior):
    detection with the pyramids, then tracking (its coarsest-level pass, the global fit and the
    tracking proper), HIP events; status counts, the error of the converged points and of their
    dense interpolation against the synthetic ground truth, beside the plain tracker's."""
    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    w = WORKLOAD
    I0n, I1n, gt, occ = synth.driving_1242x375()
    dev = torch.device("cuda", 0)
    I0, I1 = torch.from_numpy(I0n).to(dev), torch.from_numpy(I1n).to(dev)
    N = dgf.detect_count(w["W"], w["H"], w["window"], w["stride"])
    pts = torch.empty((N, 2), dtype=torch.float32, device=dev)
    flow = torch.empty((N, 2), dtype=torch.float32, device=dev)
    status = torch.empty(N, dtype=torch.uint8, device=dev)
    ws = torch.empty(dgf.track_workspace_bytes(w["W"], w["H"], w["levels"], 0), dtype=torch.uint8, device=dev)
    opts = dgf.TrackOpts(illum=True, cross=True, global_motion=True)

    def step():
        dgf.detect_pyramids(I0, I1, w["window"], w["stride"], w["levels"], ws, pts)
        e0.record()
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, opts=opts)
        e1.record()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    tt, ts = [], []
    for _ in range(steps):
        s0 = torch.cuda.Event(enable_timing=True)
        s0.record()
        step()
        torch.cuda.synchronize()
        tt.append(e0.elapsed_time(e1))
        ts.append(s0.elapsed_time(e1))
    P, F, S = pts.cpu().numpy(), flow.cpu().numpy(), status.cpu().numpy()
    conv = S == 0
    xi = np.clip(np.rint(P[conv, 0]).astype(np.int64), 0, w["W"] - 1)
    yi = np.clip(np.rint(P[conv, 1]).astype(np.int64), 0, w["H"] - 1)
    sparse_err = np.linalg.norm(F[conv] - gt[yi, xi], axis=-1)
    dense = dgf.epic(I0, pts, flow, status).cpu().numpy().astype(np.float64)
    err = np.linalg.norm(dense - gt, axis=-1)[~occ]
    out = {"workload": "driving_1242x375, illumination model + cross-based supports + global prior",
           "points": N, "ms_per_step": float(np.median(ts)), "track_ms": float(np.median(tt)),
           "points_per_s": N / (float(np.median(ts)) * 1e-3),
           "status_counts": np.bincount(S, minlength=4).tolist(),
           "seed_epe_px": float(sparse_err.mean()), "seed_median_err_px": float(np.median(sparse_err)),
           "dense_epe_noc_px": float(err.mean()), "dense_outliers_3px_noc": float((err > 3.0).mean())}
    if plain:
        out["plain"] = plain
    # each option on its own (status counts and the converged points' error, untimed)
    variants = {}
    for name, o in (("global_motion", dgf.TrackOpts(global_motion=True)), ("cross", dgf.TrackOpts(cross=True)),
                    ("illum", dgf.TrackOpts(illum=True))):
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, opts=o)
        F, S = flow.cpu().numpy(), status.cpu().numpy()
        ok = S == 0
        e = np.linalg.norm(F[ok] - gt[np.clip(np.rint(P[ok, 1]).astype(np.int64), 0, w["H"] - 1),
                                      np.clip(np.rint(P[ok, 0]).astype(np.int64), 0, w["W"] - 1)], axis=-1)
        variants[name] = {"status_counts": np.bincount(S, minlength=4).tolist(), "seed_epe_px": float(e.mean()),
                          "seeds_within_1px": int((e < 1.0).sum())}
    out["single_options"] = variants
    return out


def oracle_timings(budget_s: float):
    """The FP64 oracle on the host cores beside the GPU workloads: the small translation pair
    (median of 5), one pair of each size of the 64-pair batch, the differentiation crop (forward
    and gradient, median of 5) and a strided sample of one density-stress pair (1 run), each as
    points per second.  Bounded: every entry is a sample of a few seconds at most."""
    import numpy as np

    import oracle
    from paper_1901_09971_amd import synth

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    thr = min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores)
    res = {"threads": thr}
    c = C1
    I0, I1, _ = synth.translation_256x128()
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        pts = oracle.detect(I0, c["window"], c["stride"], threads=thr)[0]
        oracle.track(I0, I1, pts, c["levels"], c["support"], c["iters"], threads=thr)
        ts.append(time.perf_counter() - t0)
    res["translation_256x128"] = {"points": len(pts), "median_s": float(np.median(ts)),
                                  "points_per_s": len(pts) / float(np.median(ts)), "runs": 5}
    # one pair of each size of the 64-pair set (pairs 0-3), detect + track, one run
    strides = np.random.default_rng(0).choice([3, 5, 8], size=64)  # as synth.batch64_mixed draws them
    data = []
    for i, (W, H) in enumerate([(1242, 375), (1224, 370), (640, 480), (320, 240)]):
        a, b, _, _ = synth.layered_pair(W, H, seed=i, max_disp=150.0 * W / 1242.0)
        data.append(dict(I0=a, I1=b, stride=int(strides[i])))
    t0 = time.perf_counter()
    n = 0
    for d in data:
        p = oracle.detect(d["I0"], 9, d["stride"], threads=thr)[0]
        oracle.track(d["I0"], d["I1"], p, 5, 21, 20, threads=thr)
        n += len(p)
    el = time.perf_counter() - t0
    res["batch64_mixed_sample"] = {"sample": "pairs 0-3 (one of each size), detect + track", "points": n,
                                   "s": el, "points_per_s": n / el}
    # differentiation crop: 128x64 at (0, 0), window 9 stride 6 (200 points), forward + gradient
    I0f, I1f, gt = synth.translation_f32_1242x375()
    a0, a1 = np.ascontiguousarray(I0f[:64, :128]), np.ascontiguousarray(I1f[:64, :128])
    u8 = np.clip(np.rint(a0), 0, 255).astype(np.uint8)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        p = oracle.detect(u8, 9, 6, threads=thr)[0]
        f, st = oracle.track(a0, a1, p, 3, 9, 10, threads=thr)
        df = np.where((st == 0)[:, None], 2.0 * (f - np.asarray(gt, np.float64)), 0.0)
        oracle.track_grad(a0, a1, p, 9, f, st, df)
        ts.append(time.perf_counter() - t0)
    res["differentiation_crop_128x64"] = {"points": len(p), "median_s": float(np.median(ts)),
                                          "points_per_s": len(p) / float(np.median(ts)), "runs": 5,
                                          "what": "detect + track + implicit gradient (FP64)"}
    # density stress: every 64th point of pair 0, one run
    D0, D1, _, _ = synth.density_2048x1024(0)
    t0 = time.perf_counter()
    p = oracle.detect(D0, 9, 2, threads=thr)[0]
    t_det = time.perf_counter() - t0
    sub = np.ascontiguousarray(p[::64])
    t1 = time.perf_counter()
    oracle.track(D0, D1, sub, 6, 21, 20, threads=thr)
    t_trk = time.perf_counter() - t1
    res["density_2048x1024_sample"] = {"sample": f"detect all {len(p)} windows of pair 0, track every 64th point "
                                                 f"({len(sub)}), one run",
                                       "detect_s": t_det, "track_s": t_trk,
                                       "track_points_per_s": len(sub) / t_trk,
                                       "detect_points_per_s": len(p) / t_det}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-pair batched vs plain measurement")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in launch-shape heuristic")
    ap.add_argument("--batch-reps", type=int, default=10)
    ap.add_argument("--no-density", action="store_true", help="skip the 4 x 2048x1024 density stress")
    ap.add_argument("--no-illum", action="store_true", help="skip the illumination-model measurement")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation measurement")
    ap.add_argument("--density-reps", type=int, default=3)
    ap.add_argument("--no-interp", action="store_true", help="skip the dense interpolation measurement")
    ap.add_argument("--no-c1", action="store_true", help="skip the small translation pair")
    ap.add_argument("--no-imgm", action="store_true", help="skip the RLOF(IM-GM) measurement")
    ap.add_argument("--no-oracle-timings", action="store_true",
                    help="skip the oracle samples of the other workloads (the benchmark pair's stays)")
    ap.add_argument("--separate-detect", action="store_true",
                    help="step as three launches (detect, pyramids, track) instead of detect+pyramids, track")
    ap.add_argument("--no-peaks", action="store_true", help="skip the achievable-peak probes")
    ap.add_argument("--peaks-only", action="store_true", help="only run the achievable-peak probes")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the tracker shards by pairs or point ranges with no "
              "exchange in the forward pass, and the benchmark runs on a single MI355X (use --gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
        return
    if args.peaks_only:
        print(json.dumps({"achievable": achievable_peaks()}))
        return

    import numpy as np
    import torch

    import paper_1901_09971_amd as dgf
    from paper_1901_09971_amd import synth

    peaks = None if args.no_peaks else achievable_peaks()
    w = WORKLOAD
    I0n, I1n, _, _ = synth.driving_1242x375()
    dev = torch.device("cuda", 0)
    I0 = torch.from_numpy(I0n).to(dev)
    I1 = torch.from_numpy(I1n).to(dev)
    N = dgf.detect_count(w["W"], w["H"], w["window"], w["stride"])
    pts = torch.empty((N, 2), dtype=torch.float32, device=dev)
    flow = torch.empty((N, 2), dtype=torch.float32, device=dev)
    status = torch.empty(N, dtype=torch.uint8, device=dev)
    its = torch.empty(N, dtype=torch.int32, device=dev)
    ws = torch.empty(dgf.track_workspace_bytes(w["W"], w["H"], w["levels"], 0), dtype=torch.uint8, device=dev)

    # launch shape: autotuned on this pair (about a hundred timed launches, well under a second)
    tuning = None
    if not args.no_autotune:
        pts0 = dgf.detect(I0, w["window"], w["stride"])
        tuning = dgf.autotune(I0, I1, pts0, w["levels"], w["support"], w["iters"])
    else:
        tuning = dgf.get_tuning(w["support"], w["levels"], 0, N)

    fused = not args.separate_detect

    def front():
        if fused:
            dgf.detect_pyramids(I0, I1, w["window"], w["stride"], w["levels"], ws, pts)
        else:
            dgf.detect(I0, w["window"], w["stride"], out=pts)
            dgf.track_pyramids(I0, I1, w["levels"], ws)

    def step(iters_out=None):
        front()
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status, iters_out)

    # work accounting (not timed): executed iterations of every point
    step(its)
    torch.cuda.synchronize()
    it_total = int(its.to(torch.int64).sum().item())
    pix_iters = it_total * w["support"] ** 2
    st_counts = np.bincount(status.cpu().numpy(), minlength=4).tolist()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    K = args.steps
    # two events per step, around the tracking launch (each event record costs the GPU a few
    # microseconds, so the timed steps carry no others); the front end is timed as the interval
    # from one step's tracking end to the next one's start, launch gaps included
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(K)]
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host0 = time.perf_counter()
    start.record()
    for k in range(K):
        e = ev[k]
        front()
        e[0].record()
        dgf.track_run(I0, I1, pts, w["levels"], w["support"], w["iters"], ws, flow, status)
        e[1].record()
    end.record()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host0
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / K
    t_track = sum(e[0].elapsed_time(e[1]) for e in ev) / K
    t_front = (start.elapsed_time(ev[0][0]) + sum(ev[k - 1][1].elapsed_time(ev[k][0]) for k in range(1, K))) / K
    step_ms = [start.elapsed_time(ev[0][1])] + [ev[k - 1][1].elapsed_time(ev[k][1]) for k in range(1, K)]
    ms_median = float(np.median(step_ms))

    flops = pix_iters * FLOPS_PER_PIXEL_ITER
    achieved = flops / (t_track * 1e-3) / 1e12
    traffic = counter_traffic()
    fbytes = front_bytes(w["W"], w["H"], w["levels"], N)
    kname = track_kernel_name(tuning, w["support"])
    k_front = roof("hbm", fbytes, t_front, peaks)
    k_front.update({"what": ("detection beside both pyramids, one launch (k_front_u8) and the chain launch of the "
                             "last level" if fused else "detection, then both pyramids"),
                    "timed_as": "previous tracking end to tracking start (launch gaps included)",
                    "chain_launches": (w["levels"] + 2) // 4})
    k_track = roof("alu", flops, t_track, peaks, pix_iters)
    k_track.update({"kernel": kname, "iterations": it_total, "status_counts": st_counts, "tuning": tuning})
    c2_kernels = {"front": k_front, "track": k_track}
    out = {
        "metric": METRIC,
        "value": N / (ms_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": ms_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "width": w["W"], "height": w["H"], "window": w["window"],
                   "stride": w["stride"], "points": N, "levels": w["levels"], "support": w["support"],
                   "max_iters": w["iters"], "input": "uint8 pair, layered affine motion up to 150 px"},
        "roofline": {
            "bound": "alu",
            "kernel": kname,
            "achieved": achieved,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU_TFLOPS,
            "traffic": (traffic["fetch_bytes_per_launch"] + traffic["write_bytes_per_launch"]) if traffic else None,
            "algorithmic_flops_per_launch": flops,
            "pixel_iterations_per_launch": pix_iters,
            "track_ms": t_track,
            "frac_of_achievable": k_track.get("frac_achievable"),
            "issue_frac": k_track["issue_frac_nominal"],
        },
        "achievable": peaks,
        "kernels": {"driving_1242x375": dict(c2_kernels, sigma_roofline=sigma_roofline(c2_kernels, ms_step))},
        "host_wall_s": t_host,
    }
    if not args.no_c1:
        out["kernels"]["translation_256x128"] = c1_step(args.steps, args.warmup, peaks)
    if not args.no_batch:
        out["batched"] = batched_vs_plain(args.batch_reps, peaks)
    if not args.no_illum:
        out["illumination"] = illumination(args.steps, args.warmup)
    if not args.no_diff:
        out["differentiation"] = differentiation(args.steps)
    if not args.no_density:
        out["density"] = density_stress(args.density_reps, peaks)
    plain_acc = None
    if not args.no_interp:
        out["interpolation"] = interpolation(max(3, min(args.steps, 20)))
        plain_acc = {"status_counts": st_counts, "seed_epe_px": out["interpolation"]["seed_epe_px"],
                     "dense_epe_noc_px": out["interpolation"]["epe_noc_px"],
                     "dense_outliers_3px_noc": out["interpolation"]["outliers_3px_noc"]}
    if not args.no_imgm:
        out["rlof_im_gm"] = im_gm(max(5, min(args.steps, 20)), 3, plain_acc)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I0n, I1n, N, args.cpu_budget_s, interp=not args.no_interp)
        out["cpu_baseline"].update(lscpu_info())
        if not args.no_oracle_timings:
            out["cpu_baseline"]["other_workloads"] = oracle_timings(args.cpu_budget_s)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
