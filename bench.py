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
runs on.  ``cpu_baseline`` times the FP64 CPU oracle on the same pair on the host cores.
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


def cpu_baseline(I0, I1, n_points, budget_s, seeds=None):
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
        oracle.track(I0, I1, pts, w["levels"], w["support"], w["iters"], threads=threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 3:
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
    if seeds is not None:
        # the dense interpolation of the GPU-tracked points of the same pair (geodesic partition
        # single-threaded, neighbour searches and fits over the host threads)
        P, F, S = seeds
        t2 = time.perf_counter()
        oracle.epic(I0, P.astype(np.float64), F.astype(np.float64), S)
        res["interpolation_s"] = time.perf_counter() - t2
    return res


def batched_vs_plain(reps: int):
    """Frame-pairs/s on the 64-pair mixed set (four sizes, strides 3/5/8; 5 levels, 21x21, 20
    iterations): per-pair launches (detect, 4 pyramid levels, track for each pair in turn) vs one
    replay of the captured batched plan.  Same tracker launch shape in both."""
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
    # the two forms must agree exactly
    P = torch.cat([B["p"] for B in bufs])
    S = torch.cat([B["s"] for B in bufs])
    identical = bool(torch.equal(P, plan.points) and torch.equal(S, plan.status))
    npts = plan.num_points
    plan.close()
    return {"pairs": len(pairs), "points": npts, "reps": reps,
            "plain_ms": t_plain, "batched_ms": t_batch,
            "plain_pairs_per_s": len(pairs) / (t_plain * 1e-3),
            "batched_pairs_per_s": len(pairs) / (t_batch * 1e-3),
            "speedup": t_plain / t_batch, "identical_outputs": identical,
            "batched_track_tflops_lower_bound": pix_iters * FLOPS_PER_PIXEL_ITER / (t_batch * 1e-3) / 1e12,
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
    (its geodesic relaxation runs to a fixed point), so it is timed on the host clock.  Accuracy:
    endpoint error and > 3 px rate of the dense field on the non-occluded pixels of the synthetic
    ground truth.  Also returns the points, flows and statuses it interpolated."""
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
            "seed_epe_px": float(sparse_err.mean())}, (P, F, S)


DENSITY = dict(name="density_2048x1024x4", W=2048, H=1024, pairs=4, window=9, stride=2, levels=6, support=21,
               iters=20)


def density_stress(reps: int):
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
    return {"workload": c["name"], "pairs": c["pairs"], "points": n, "levels": c["levels"],
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
    ap.add_argument("--separate-detect", action="store_true",
                    help="step as three launches (detect, pyramids, track) instead of detect+pyramids, track")
    ap.add_argument("--no-peaks", action="store_true", help="skip the achievable-peak probes")
    ap.add_argument("--peaks-only", action="store_true", help="only run the achievable-peak probes")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the tracker shards by pairs or point ranges with no "
              "exchange in the forward pass, and this build runs on a single MI355X (use --gpus 1).",
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
    det_bytes = w["W"] * w["H"] + 8 * N
    pyr_read = pyr_write = 0
    Wl, Hl = w["W"], w["H"]
    for _ in range(w["levels"] - 1):
        pyr_read += 2 * Wl * Hl
        Wl, Hl = (Wl + 1) // 2, (Hl + 1) // 2
        pyr_write += 2 * Wl * Hl
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
            "kernel": "k_track",
            "achieved": achieved,
            "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VALU_TFLOPS,
            "traffic": (traffic["fetch_bytes_per_launch"] + traffic["write_bytes_per_launch"]) if traffic else None,
            "algorithmic_flops_per_launch": flops,
            "pixel_iterations_per_launch": pix_iters,
            "track_ms": t_track,
        },
        "kernels": {
            "front": {"ms": t_front, "what": ("detection beside both pyramids, one launch" if fused else
                                              "detection, then both pyramids: two launches"),
                      "timed_as": "previous tracking end to tracking start (launch gaps included)",
                      "chain_launches": (w["levels"] + 2) // 4,
                      "algorithmic_bytes": pyr_read + pyr_write + det_bytes,
                      "hbm_frac": (pyr_read + pyr_write + det_bytes) / (t_front * 1e-3) / (PEAK_HBM_GBPS * 1e9)},
            "track": {"ms": t_track, "iterations": it_total, "status_counts": st_counts, "tuning": tuning},
        },
        "host_wall_s": t_host,
    }
    if not args.no_batch:
        out["batched"] = batched_vs_plain(args.batch_reps)
    if not args.no_illum:
        out["illumination"] = illumination(args.steps, args.warmup)
    if not args.no_diff:
        out["differentiation"] = differentiation(args.steps)
    if not args.no_density:
        out["density"] = density_stress(args.density_reps)
    seeds = None
    if not args.no_interp:
        out["interpolation"], seeds = interpolation(max(3, min(args.steps, 20)))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I0n, I1n, N, args.cpu_budget_s, seeds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
