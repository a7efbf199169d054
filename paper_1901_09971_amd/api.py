"""PyTorch-facing binding of the C ABI: tensors supply device memory and the current stream;
every step of detection and tracking runs in the HIP library."""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import DGF_F32, DGF_TRACK_CROSS, DGF_TRACK_GLOBAL, DGF_TRACK_ILLUM, DGF_U8, DgfEpicOpts, DgfImage, DgfTrackOpts, check, lib


@dataclass
class TrackOpts:
    """Robust tracker constants (0..255 intensity scale); see dgf_track_opts in the C header."""
    sigma1: float = 8.0
    sigma2: float = 32.0
    eps_coarse: float = 1e-2
    eps_fine: float = 1e-4
    min_eig: float = 1e-4 * 255.0 * 255.0
    illum: bool = False  # per-point gain and offset estimated with the flow (DGF_TRACK_ILLUM)
    cross: bool = False  # adaptive cross-based supports (DGF_TRACK_CROSS)
    global_motion: bool = False  # global affine prior for the coarsest level (DGF_TRACK_GLOBAL)
    cross_tau: float = 25.0  # arm threshold of the cross-based supports, intensity units

    def flags(self) -> int:
        return ((DGF_TRACK_ILLUM if self.illum else 0) | (DGF_TRACK_CROSS if self.cross else 0)
                | (DGF_TRACK_GLOBAL if self.global_motion else 0))

    def to_c(self) -> DgfTrackOpts:
        return DgfTrackOpts(self.sigma1, self.sigma2, self.eps_coarse, self.eps_fine, self.min_eig, self.flags(),
                            self.cross_tau)


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _image(t: torch.Tensor, name: str) -> DgfImage:
    if not isinstance(t, torch.Tensor) or t.dim() != 2:
        raise ValueError(f"{name}: expected a 2-D tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device (cuda) tensor")
    if t.dtype == torch.uint8:
        dt = DGF_U8
    elif t.dtype == torch.float32:
        dt = DGF_F32
    else:
        raise ValueError(f"{name}: dtype must be uint8 or float32")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        raise ValueError(f"{name}: rows must be contiguous")
    return DgfImage(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0) * t.element_size(), dt)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def detect_count(width: int, height: int, window: int, stride: int) -> int:
    return int(lib().dgf_detect_count(width, height, window, stride))


def detect(frame: torch.Tensor, window: int, stride: int, return_sel: bool = False,
           return_response: bool = False, out: torch.Tensor | None = None):
    """DeGraF key-points of a uint8 frame: float32 [N, 2] (x, y) in row-major window order.
    ``out`` (float32 [N, 2] device) receives the points instead of a new tensor."""
    img = _image(frame, "frame")
    n = detect_count(img.width, img.height, window, stride)
    if n < 0:
        raise ValueError("window and stride must be >= 1")
    if out is not None:
        if out.shape != (n, 2) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out: expected a contiguous float32 [N, 2] tensor")
        pts = out
    else:
        pts = torch.empty((n, 2), dtype=torch.float32, device=frame.device)
    sel = torch.empty(n, dtype=torch.uint8, device=frame.device) if return_sel else None
    resp = torch.empty(n, dtype=torch.float32, device=frame.device) if return_response else None
    check(lib().dgf_detect(ctypes.byref(img), window, stride, _ptr(pts), _ptr(sel), _ptr(resp), n, _stream()),
          "dgf_detect")
    out = [pts]
    if return_sel:
        out.append(sel)
    if return_response:
        out.append(resp)
    return out[0] if len(out) == 1 else tuple(out)


def pyramid_layout(width: int, height: int, levels: int, dtype: int):
    off = (ctypes.c_int64 * _lib.DGF_MAX_LEVELS)()
    pit = (ctypes.c_int64 * _lib.DGF_MAX_LEVELS)()
    total = int(lib().dgf_pyramid_layout(width, height, levels, dtype, off, pit))
    return total, list(off)[:levels], list(pit)[:levels]


def pyramid(img: torch.Tensor, levels: int):
    """Levels 0 .. levels-1 (level 0 is ``img``); coarser levels are views into one buffer."""
    im = _image(img, "img")
    total, off, pit = pyramid_layout(im.width, im.height, levels, im.dtype)
    buf = torch.empty(max(total, 1), dtype=torch.uint8, device=img.device)
    check(lib().dgf_pyramid(ctypes.byref(im), levels, _ptr(buf), total, _stream()), "dgf_pyramid")
    out = [img]
    W, H = im.width, im.height
    esz = img.element_size()
    for l in range(1, levels):
        W, H = (W + 1) // 2, (H + 1) // 2
        rows = buf[off[l]:off[l] + pit[l] * H].view(H, pit[l])
        lvl = rows[:, :W * esz]
        out.append(lvl if esz == 1 else lvl.contiguous().view(torch.float32))
    return out


def track_workspace_bytes(width: int, height: int, levels: int, dtype: int) -> int:
    return int(lib().dgf_track_workspace_bytes(width, height, levels, dtype))


def track(I0: torch.Tensor, I1: torch.Tensor, points: torch.Tensor, levels: int, support: int, iters: int,
          opts: TrackOpts | None = None, return_iters: bool = False, workspace: torch.Tensor | None = None,
          return_illum: bool = False, return_gm: bool = False):
    """Track ``points`` (float32 [n, 2] device) from I0 to I1.  Returns (flow float32 [n, 2],
    status uint8 [n]), then the per-point iteration count (int32 [n]) if ``return_iters``, the
    per-point (gain m, offset c) (float32 [n, 2], needs ``opts.illum``) if ``return_illum`` and the
    fitted global affine motion (float64 [2, 3] device, needs ``opts.global_motion``) if
    ``return_gm``."""
    if return_gm and not (opts is not None and opts.global_motion):
        raise ValueError("return_gm needs opts.global_motion")
    a, b = _image(I0, "I0"), _image(I1, "I1")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 2 or not points.is_cuda:
        raise ValueError("points: expected a float32 [n, 2] device tensor")
    points = points.contiguous()
    n = points.shape[0]
    ws_bytes = track_workspace_bytes(a.width, a.height, levels, a.dtype)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=I0.device)
    flow = torch.empty((n, 2), dtype=torch.float32, device=I0.device)
    status = torch.empty(n, dtype=torch.uint8, device=I0.device)
    its = torch.empty(n, dtype=torch.int32, device=I0.device) if return_iters else None
    ill = torch.empty((n, 2), dtype=torch.float32, device=I0.device) if return_illum else None
    o = (opts or TrackOpts()).to_c()
    check(lib().dgf_track(ctypes.byref(a), ctypes.byref(b), _ptr(points), n, levels, support, iters,
                          ctypes.byref(o), _ptr(workspace), workspace.numel(), _ptr(flow), _ptr(status), _ptr(its),
                          _ptr(ill), _stream()), "dgf_track")
    out = (flow, status)
    if return_iters:
        out += (its,)
    if return_illum:
        out += (ill,)
    if return_gm:
        # the model sits right after both pyramids in the workspace
        at = 2 * pyramid_layout(a.width, a.height, levels, a.dtype)[0]
        out += (workspace[at:at + 48].clone().view(torch.float64).view(2, 3),)
    return out


def gm_fit(points: torch.Tensor, flow: torch.Tensor, status: torch.Tensor, width: int, height: int,
           scale: float) -> torch.Tensor:
    """Robust global affine motion (float64 [2, 3] device, v = A (x - (width-1)/2, y - (height-1)/2,
    1)) of the converged points of a tracking result (dgf_gm_fit; Tukey scale ``scale`` pixels)."""
    n = points.shape[0]
    for t, shape, dt, name in ((points, (n, 2), torch.float32, "points"), (flow, (n, 2), torch.float32, "flow"),
                               (status, (n,), torch.uint8, "status")):
        if t.shape != shape or t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {dt} device tensor of shape {shape}")
    ws = torch.empty(int(lib().dgf_gm_workspace_bytes()), dtype=torch.uint8, device=points.device)
    model = torch.empty((2, 3), dtype=torch.float64, device=points.device)
    check(lib().dgf_gm_fit(_ptr(points), _ptr(flow), _ptr(status), n, width, height, float(scale), _ptr(ws),
                           ws.numel(), _ptr(model), _stream()), "dgf_gm_fit")
    return model


def track_static(I0: torch.Tensor, I1: torch.Tensor, points: torch.Tensor, levels: int, support: int, iters: int,
                 opts: TrackOpts | None = None, return_iters: bool = False, return_illum: bool = False):
    """``track`` through ``dgf_track_static``: the pyramids go to the library's per-GPU static
    scratch array instead of a workspace (the call allocates no device memory; outputs are
    allocated here, by the caller of the C entry point).  Calls overlapping on one GPU race."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 2 or not points.is_cuda:
        raise ValueError("points: expected a float32 [n, 2] device tensor")
    points = points.contiguous()
    n = points.shape[0]
    flow = torch.empty((n, 2), dtype=torch.float32, device=I0.device)
    status = torch.empty(n, dtype=torch.uint8, device=I0.device)
    its = torch.empty(n, dtype=torch.int32, device=I0.device) if return_iters else None
    ill = torch.empty((n, 2), dtype=torch.float32, device=I0.device) if return_illum else None
    o = (opts or TrackOpts()).to_c()
    check(lib().dgf_track_static(ctypes.byref(a), ctypes.byref(b), _ptr(points), n, levels, support, iters,
                                 ctypes.byref(o), _ptr(flow), _ptr(status), _ptr(its), _ptr(ill), _stream()),
          "dgf_track_static")
    out = (flow, status)
    if return_iters:
        out += (its,)
    if return_illum:
        out += (ill,)
    return out


def track_pyramids(I0: torch.Tensor, I1: torch.Tensor, levels: int, workspace: torch.Tensor) -> None:
    """First stage of :func:`track`: build both pyramids into ``workspace`` (uint8 device
    tensor of at least track_workspace_bytes(...) bytes)."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    check(lib().dgf_track_pyramids(ctypes.byref(a), ctypes.byref(b), levels, _ptr(workspace), workspace.numel(),
                                   _stream()), "dgf_track_pyramids")


def detect_pyramids(I0: torch.Tensor, I1: torch.Tensor, window: int, stride: int, levels: int,
                    workspace: torch.Tensor, points: torch.Tensor, sel: torch.Tensor | None = None,
                    response: torch.Tensor | None = None) -> None:
    """:func:`detect` on ``I0`` into ``points`` (float32 [n, 2], n = :func:`detect_count`; optional
    ``sel`` uint8 [n] and ``response`` float32 [n]) and :func:`track_pyramids` of the pair into
    ``workspace``, in one launch where they fit one (dgf_detect_pyramids)."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    n = detect_count(I0.shape[1], I0.shape[0], window, stride)
    if points.shape != (n, 2) or points.dtype != torch.float32 or not points.is_contiguous():
        raise ValueError(f"points: expected a contiguous float32 tensor of shape {(n, 2)}")
    for t, dt, name in ((sel, torch.uint8, "sel"), (response, torch.float32, "response")):
        if t is not None and (t.shape != (n,) or t.dtype != dt or not t.is_contiguous()):
            raise ValueError(f"{name}: expected a contiguous {dt} tensor of shape {(n,)}")
    check(lib().dgf_detect_pyramids(ctypes.byref(a), ctypes.byref(b), window, stride, levels, _ptr(workspace),
                                    workspace.numel(), _ptr(points), _ptr(sel), _ptr(response), n, _stream()),
          "dgf_detect_pyramids")


def track_run(I0: torch.Tensor, I1: torch.Tensor, points: torch.Tensor, levels: int, support: int, iters: int,
              workspace: torch.Tensor, flow: torch.Tensor, status: torch.Tensor, iters_out: torch.Tensor | None = None,
              opts: TrackOpts | None = None, illum_out: torch.Tensor | None = None) -> None:
    """Second stage of :func:`track` on pyramids already built by :func:`track_pyramids`;
    writes into the caller's ``flow`` (float32 [n, 2]) and ``status`` (uint8 [n]), and the
    per-point (gain, offset) into ``illum_out`` (float32 [n, 2], with ``opts.illum``) when given."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    n = points.shape[0]
    if flow.shape != (n, 2) or flow.dtype != torch.float32 or status.shape != (n,) or status.dtype != torch.uint8:
        raise ValueError("flow/status: wrong shape or dtype")
    if illum_out is not None and (illum_out.shape != (n, 2) or illum_out.dtype != torch.float32
                                  or not illum_out.is_contiguous()):
        raise ValueError("illum_out: expected a contiguous float32 [n, 2] tensor")
    o = (opts or TrackOpts()).to_c()
    check(lib().dgf_track_run(ctypes.byref(a), ctypes.byref(b), _ptr(points), n, levels, support, iters,
                              ctypes.byref(o), _ptr(workspace), workspace.numel(), _ptr(flow), _ptr(status),
                              _ptr(iters_out), _ptr(illum_out), _stream()), "dgf_track_run")


def track_backward(I0: torch.Tensor, I1: torch.Tensor, points: torch.Tensor, support: int, flow: torch.Tensor,
                   status: torch.Tensor, dflow: torch.Tensor, dI0: torch.Tensor, dI1: torch.Tensor,
                   opts: TrackOpts | None = None, dpoints: torch.Tensor | None = None,
                   illum: torch.Tensor | None = None) -> None:
    """Accumulate dL/dI0 into ``dI0`` and dL/dI1 into ``dI1`` (float32, same shape and row stride
    as the images) for the upstream gradient ``dflow`` of a forward :func:`track` call; write
    dL/dp into ``dpoints`` (float32 [n, 2]) when given.  With ``opts.illum`` the forward call's
    per-point (gain, offset) go in ``illum`` (float32 [n, 2])."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    for t, ref, name in ((dI0, I0, "dI0"), (dI1, I1, "dI1")):
        if t.dtype != torch.float32 or t.shape != ref.shape or t.stride() != ref.stride() or not t.is_cuda:
            raise ValueError(f"{name}: expected float32 with the shape and strides of the image")
    n = points.shape[0]
    dflow = dflow.contiguous().to(torch.float32)
    o = (opts or TrackOpts()).to_c()
    if dpoints is not None and (dpoints.shape != (n, 2) or dpoints.dtype != torch.float32 or not dpoints.is_contiguous()):
        raise ValueError("dpoints: expected a contiguous float32 [n, 2] tensor")
    if illum is not None:
        if illum.shape != (n, 2) or illum.dtype != torch.float32:
            raise ValueError("illum: expected a float32 [n, 2] tensor")
        illum = illum.contiguous()
    check(lib().dgf_track_backward(ctypes.byref(a), ctypes.byref(b), _ptr(points.contiguous()), n, support,
                                   ctypes.byref(o), _ptr(flow.contiguous()), _ptr(status.contiguous()), _ptr(dflow),
                                   _ptr(dI0), _ptr(dI1), _ptr(dpoints), _ptr(illum), _stream()), "dgf_track_backward")


def detect_backward(frame: torch.Tensor, window: int, stride: int, sel: torch.Tensor, dpoints: torch.Tensor,
                    dI0: torch.Tensor) -> None:
    """Accumulate into ``dI0`` (float32 [H, W]) the gradient through detection of the upstream
    gradient ``dpoints`` = dL/dp (dgf_detect_backward); ``frame`` and ``sel`` as in :func:`detect`."""
    a = _image(frame, "frame")
    n = int(lib().dgf_detect_count(a.width, a.height, window, stride))
    if dI0.dtype != torch.float32 or dI0.dim() != 2 or dI0.shape != frame.shape or dI0.stride(1) != 1:
        raise ValueError("dI0: expected a float32 [H, W] tensor with unit column stride")
    dpoints = dpoints.contiguous().to(torch.float32)
    check(lib().dgf_detect_backward(ctypes.byref(a), window, stride, _ptr(sel.contiguous()), _ptr(dpoints), n,
                                    _ptr(dI0), dI0.stride(0), _stream()), "dgf_detect_backward")


class DetectFn(torch.autograd.Function):
    """points = DetectFn.apply(I0, window, stride)

    Differentiable DeGraF detection of a float32 frame holding grey levels: the forward pass
    detects on the frame rounded to uint8, the backward pass is the gradient of the centroid
    ratios at those values (dgf_detect_backward)."""

    @staticmethod
    def forward(ctx, I0, window, stride):
        u8 = I0.detach().round().clamp(0, 255).to(torch.uint8)
        points, sel = detect(u8, window, stride, return_sel=True)
        ctx.save_for_backward(u8, sel)
        ctx.window, ctx.stride = window, stride
        return points

    @staticmethod
    def backward(ctx, dpoints):
        u8, sel = ctx.saved_tensors
        dI0 = torch.zeros(u8.shape, dtype=torch.float32, device=u8.device)
        if dpoints is not None:
            detect_backward(u8, ctx.window, ctx.stride, sel, dpoints, dI0)
        return dI0, None, None


class TrackFn(torch.autograd.Function):
    """flow, status = TrackFn.apply(I0, I1, points, levels, support, iters, opts)

    Differentiable tracking of float32 frames: the backward pass is the implicit-function adjoint
    at the converged level-0 fixed point (dgf_track_backward), w.r.t. both frames and the point
    positions; points that did not converge get no gradient.  With ``opts.illum`` the adjoint
    is that of the illumination model."""

    @staticmethod
    def forward(ctx, I0, I1, points, levels, support, iters, opts=None):
        im = bool(opts is not None and opts.illum)
        if im:
            flow, status, ill = track(I0, I1, points, levels, support, iters, opts=opts, return_illum=True)
        else:
            (flow, status), ill = track(I0, I1, points, levels, support, iters, opts=opts), None
        ctx.save_for_backward(I0, I1, points, flow, status, ill)
        ctx.support = support
        ctx.opts = opts
        ctx.mark_non_differentiable(status)
        return flow, status

    @staticmethod
    def backward(ctx, dflow, _dstatus):
        I0, I1, points, flow, status, ill = ctx.saved_tensors
        dI0 = torch.zeros_like(I0)
        dI1 = torch.zeros_like(I1)
        dpoints = torch.zeros_like(points) if ctx.needs_input_grad[2] else None
        if dflow is not None:
            track_backward(I0, I1, points, ctx.support, flow, status, dflow, dI0, dI1, ctx.opts, dpoints, ill)
        return dI0, dI1, dpoints, None, None, None, None


@dataclass
class EpicOpts:
    """Interpolation constants; see dgf_epic_opts in the C header."""
    k: int = 128
    kappa: int = 8
    half_dist: int = 64

    def to_c(self) -> DgfEpicOpts:
        return DgfEpicOpts(self.k, self.kappa, self.half_dist)


def epic_workspace_bytes(width: int, height: int, n: int) -> int:
    return int(lib().dgf_epic_workspace_bytes(width, height, n))


def _epic_buffers(frame, points, flow, status, opts, return_aux, workspace, dense):
    a = _image(frame, "frame")
    if a.dtype != DGF_U8:
        raise ValueError("frame: expected uint8")
    n = points.shape[0]
    for t, name, dt in ((points, "points", torch.float32), (flow, "flow", torch.float32)):
        if t.dtype != dt or t.shape != (n, 2) or not t.is_cuda:
            raise ValueError(f"{name}: expected a float32 [n, 2] device tensor")
    if status.dtype != torch.uint8 or status.shape != (n,) or not status.is_cuda:
        raise ValueError("status: expected a uint8 [n] device tensor")
    o = opts or EpicOpts()
    H, W = frame.shape
    ws_bytes = epic_workspace_bytes(W, H, n)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=frame.device)
    if dense is None:
        dense = torch.empty((H, W, 2), dtype=torch.float32, device=frame.device)
    elif dense.shape != (H, W, 2) or dense.dtype != torch.float32 or not dense.is_contiguous():
        raise ValueError("dense: expected a contiguous float32 [H, W, 2] tensor")
    aux = None
    if return_aux:
        dev = frame.device
        aux = dict(labels=torch.empty((H, W), dtype=torch.int32, device=dev),
                   dist=torch.empty((H, W), dtype=torch.int32, device=dev),  # holds uint32 bits
                   nbr=torch.empty((n, o.k), dtype=torch.int32, device=dev),
                   nbr_dist=torch.empty((n, o.k), dtype=torch.int32, device=dev),  # uint32 bits
                   model=torch.empty((n, 6), dtype=torch.float32, device=dev))
    g = (lambda key: _ptr(aux[key])) if aux else (lambda key: None)
    args = (ctypes.byref(a), _ptr(points.contiguous()), _ptr(flow.contiguous()), _ptr(status.contiguous()), n,
            ctypes.byref(o.to_c()), _ptr(workspace), workspace.numel(), _ptr(dense), 2 * W, g("labels"), g("dist"),
            g("nbr"), g("nbr_dist"), g("model"))
    return args, dense, aux


def epic(frame: torch.Tensor, points: torch.Tensor, flow: torch.Tensor, status: torch.Tensor,
         opts: EpicOpts | None = None, return_aux: bool = False, workspace: torch.Tensor | None = None):
    """Dense flow float32 [H, W, 2] of the uint8 ``frame`` interpolated from the tracked ``points``
    (float32 [n, 2]) with their ``flow`` and ``status`` (dgf_epic).  With ``return_aux`` also a dict
    of labels and dist [H, W], nbr and nbr_dist [n, k] and model [n, 6].  Synchronises the stream."""
    args, dense, aux = _epic_buffers(frame, points, flow, status, opts, return_aux, workspace, None)
    check(lib().dgf_epic(*args, _stream()), "dgf_epic")
    if return_aux:
        return dense, aux
    return dense


def epic_async(frame: torch.Tensor, points: torch.Tensor, flow: torch.Tensor, status: torch.Tensor,
               opts: EpicOpts | None = None, max_relax: int = 0, return_aux: bool = False,
               workspace: torch.Tensor | None = None, dense: torch.Tensor | None = None,
               status_out: torch.Tensor | None = None):
    """:func:`epic` without synchronising the stream (dgf_epic_async), so it can be captured in a
    graph: ``max_relax`` geodesic relaxation launches (0 = the library default).  Returns
    (dense, status_out[, aux]); status_out, an int32 [1] device tensor, holds 0 when done, 1 when
    the relaxation needed more launches (nothing written), 2 on a capacity limit."""
    args, dense, aux = _epic_buffers(frame, points, flow, status, opts, return_aux, workspace, dense)
    if status_out is None:
        status_out = torch.empty(1, dtype=torch.int32, device=frame.device)
    elif status_out.dtype != torch.int32 or status_out.numel() < 1 or not status_out.is_cuda:
        raise ValueError("status_out: expected an int32 device tensor")
    check(lib().dgf_epic_async(*args, int(max_relax), _ptr(status_out), _stream()), "dgf_epic_async")
    if return_aux:
        return dense, status_out, aux
    return dense, status_out


def _tuning_dict(t) -> dict:
    return dict(lanes_per_point=t.lanes_per_point, waves_per_group=t.waves_per_group, margin=t.margin,
                kernel=t.kernel, ms=t.ms)


def get_tuning(support: int, levels: int, dtype: int = DGF_U8, n: int = 0) -> dict:
    t = _lib.DgfTuning()
    check(lib().dgf_get_tuning(support, levels, dtype, n, ctypes.byref(t)), "dgf_get_tuning")
    return _tuning_dict(t)


def set_tuning(support: int, dtype: int, lanes_per_point: int, waves_per_group: int, margin: int, kernel: int = 0):
    t = _lib.DgfTuning(lanes_per_point, waves_per_group, margin, kernel, -1.0)
    check(lib().dgf_set_tuning(support, dtype, ctypes.byref(t)), "dgf_set_tuning")


def autotune(I0: torch.Tensor, I1: torch.Tensor, points: torch.Tensor, levels: int, support: int, iters: int,
             opts: TrackOpts | None = None, cache_path: str | None = None, return_result: bool = False):
    """Time every compiled launch shape on these inputs, install the fastest for (support,
    dtype) and return it (dgf_autotune); with ``return_result`` also the (flow, status) the call
    leaves, a tracking result made with the installed shape."""
    a, b = _image(I0, "I0"), _image(I1, "I1")
    points = points.contiguous()
    n = points.shape[0]
    ws = torch.empty(max(track_workspace_bytes(a.width, a.height, levels, a.dtype), 1), dtype=torch.uint8,
                     device=I0.device)
    flow = torch.empty((n, 2), dtype=torch.float32, device=I0.device)
    status = torch.empty(n, dtype=torch.uint8, device=I0.device)
    o = (opts or TrackOpts()).to_c()
    t = _lib.DgfTuning()
    check(lib().dgf_autotune(ctypes.byref(a), ctypes.byref(b), _ptr(points), n, levels, support, iters,
                             ctypes.byref(o), _ptr(ws), ws.numel(), _ptr(flow), _ptr(status),
                             cache_path.encode() if cache_path else None, ctypes.byref(t), _stream()), "dgf_autotune")
    if return_result:
        return _tuning_dict(t), flow, status
    return _tuning_dict(t)


class Batch:
    """Plan for detect + pyramids + track of many uint8 frame pairs of uneven size in one pass
    (dgf_batch_*).  ``pairs`` is a list of (I0, I1, window, stride); the tensors are kept alive
    by the plan.  Outputs of all pairs are concatenated in pair order (see ``offsets``)."""

    def __init__(self, pairs, levels: int, support: int, iters: int, opts: TrackOpts | None = None):
        self._keep = [(a, b) for a, b, _, _ in pairs]
        descs = (_lib.DgfPairDesc * len(pairs))()
        for i, (a, b, window, stride) in enumerate(pairs):
            descs[i] = _lib.DgfPairDesc(_image(a, f"pairs[{i}].I0"), _image(b, f"pairs[{i}].I1"), window, stride)
        o = (opts or TrackOpts()).to_c()
        self.illum_model = bool(opts is not None and opts.illum)
        h = ctypes.c_void_p()
        check(lib().dgf_batch_create(descs, len(pairs), levels, support, iters, ctypes.byref(o), ctypes.byref(h)),
              "dgf_batch_create")
        self._h = h
        self.device = pairs[0][0].device
        self.num_points = int(lib().dgf_batch_num_points(h))
        off = (ctypes.c_int64 * (len(pairs) + 1))()
        check(lib().dgf_batch_point_offsets(h, off), "dgf_batch_point_offsets")
        self.offsets = list(off)
        n = self.num_points
        self.points = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        self.flow = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        self.status = torch.empty(n, dtype=torch.uint8, device=self.device)
        # per-point gain and offset of the illumination model (None for the plain model)
        self.illum = torch.empty((n, 2), dtype=torch.float32, device=self.device) if self.illum_model else None

    def run(self, iters_out: torch.Tensor | None = None):
        """Eager run on the current stream; returns (points, flow, status) views of the plan's
        buffers (with the illumination model, ``self.illum`` holds the gain and offset)."""
        check(lib().dgf_batch_run(self._h, _ptr(self.points), _ptr(self.flow), _ptr(self.status), _ptr(iters_out),
                                  _ptr(self.illum), _stream()), "dgf_batch_run")
        return self.points, self.flow, self.status

    def front(self):
        """First half of :meth:`run`: every pair's pyramids and points (into ``self.points``)."""
        check(lib().dgf_batch_front(self._h, _ptr(self.points), _stream()), "dgf_batch_front")
        return self.points

    def track(self, points: torch.Tensor | None = None, iters_out: torch.Tensor | None = None):
        """Second half of :meth:`run`: track ``points`` (default: the plan's own, as the last
        :meth:`front` detected them) on the pyramids of the last :meth:`front`."""
        p = self.points if points is None else points
        if p.shape != self.points.shape or p.dtype != torch.float32 or not p.is_contiguous():
            raise ValueError("points: expected a contiguous float32 tensor of the plan's point count")
        check(lib().dgf_batch_track(self._h, _ptr(p), _ptr(self.flow), _ptr(self.status), _ptr(iters_out),
                                    _ptr(self.illum), _stream()), "dgf_batch_track")
        return self.flow, self.status

    def capture(self):
        """Capture the run into a HIP graph on the current (non-default) stream."""
        check(lib().dgf_batch_capture(self._h, _ptr(self.points), _ptr(self.flow), _ptr(self.status),
                                      _ptr(self.illum), _stream()), "dgf_batch_capture")

    def replay(self):
        check(lib().dgf_batch_replay(self._h, _stream()), "dgf_batch_replay")
        return self.points, self.flow, self.status

    def level(self, pair: int, frame: int, level: int):
        """Where the plan keeps pyramid level ``level`` of frame ``frame`` (0 = I0, 1 = I1) of pair
        ``pair`` (dgf_batch_level): (device address, row pitch in bytes, width, height).  The
        bytes are the plan's and are rewritten by the next front or run."""
        data, pitch = ctypes.c_void_p(), ctypes.c_int64()
        w, h = ctypes.c_int32(), ctypes.c_int32()
        check(lib().dgf_batch_level(self._h, pair, frame, level, ctypes.byref(data), ctypes.byref(pitch),
                                    ctypes.byref(w), ctypes.byref(h)), "dgf_batch_level")
        return int(data.value or 0), pitch.value, w.value, h.value

    def grad_layout(self):
        """(total floats, per-pair offsets of dI0) of the buffer :meth:`backward` writes; pair i's
        dI1 follows its dI0, each a dense height x width float map."""
        off = (ctypes.c_int64 * (len(self._keep) + 1))()
        total = int(lib().dgf_batch_grad_size(self._h, off))
        return total, list(off)

    def backward(self, dflow: torch.Tensor, grad: torch.Tensor | None = None, points: torch.Tensor | None = None,
                 flow: torch.Tensor | None = None, status: torch.Tensor | None = None,
                 illum: torch.Tensor | None = None):
        """Gradient w.r.t. every pair's frames for the upstream gradient ``dflow`` (float32
        [num_points, 2]) in one launch (dgf_batch_backward), at the last run's points, flow,
        status (and gain / offset) unless others of the same shapes are given.  Returns the flat
        buffer and a list of (dI0, dI1) views, one per pair."""
        total, off = self.grad_layout()
        if grad is None or grad.numel() < total or grad.dtype != torch.float32:
            grad = torch.empty(max(total, 1), dtype=torch.float32, device=self.device)
        dflow = dflow.contiguous().to(torch.float32)
        if dflow.shape != (self.num_points, 2):
            raise ValueError("dflow: expected float32 [num_points, 2]")
        state = []
        for name, given, own in (("points", points, self.points), ("flow", flow, self.flow),
                                 ("status", status, self.status), ("illum", illum, self.illum)):
            if given is None or own is None:
                state.append(own)
                continue
            if given.shape != own.shape or given.dtype != own.dtype or not given.is_contiguous():
                raise ValueError(f"{name}: expected a contiguous {own.dtype} tensor of shape {tuple(own.shape)}")
            state.append(given)
        p, f, st, ill = state
        check(lib().dgf_batch_backward(self._h, _ptr(p), _ptr(f), _ptr(st), _ptr(dflow), _ptr(ill), _ptr(grad),
                                       _stream()), "dgf_batch_backward")
        views = []
        for i, (a, _) in enumerate(self._keep):
            H, W = a.shape
            o = off[i]
            views.append((grad[o:o + H * W].view(H, W), grad[o + H * W:o + 2 * H * W].view(H, W)))
        return grad, views

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            check(lib().dgf_batch_destroy(self._h), "dgf_batch_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass


def track_batched(pairs, levels: int, support: int, iters: int, opts: TrackOpts | None = None):
    """Detect and track many uint8 pairs of uneven size in one pass (a :class:`Batch` plan, run
    once): ``pairs`` is a list of (I0, I1, window, stride); returns one (points, flow, status)
    per pair, copies of the plan's outputs."""
    plan = Batch(pairs, levels, support, iters, opts=opts)
    try:
        P, F, S = plan.run()
        out = []
        for i in range(len(pairs)):
            lo, hi = plan.offsets[i], plan.offsets[i + 1]
            out.append((P[lo:hi].clone(), F[lo:hi].clone(), S[lo:hi].clone()))
        return out
    finally:
        plan.close()


INF = math.inf
