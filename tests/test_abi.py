"""CPU checks of the C ABI: the library loads, exports every function the header declares, and
its host-only entry points (sizes, layouts, defaults, argument validation that returns before
any launch) behave as documented.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1901_09971_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared():
    names = set()
    for f in os.listdir(HEADER_DIR):
        if f.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(dgf_[a-z0-9_]+)\s*\(", text))
    return names


def test_header_declares_and_library_exports_everything():
    declared = _declared()
    assert "dgf_detect" in declared and "dgf_track" in declared
    L = _lib.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(dgf_[a-z0-9_]+)\b", out))
    assert declared <= exported
    # the Python signature table covers exactly the declared functions
    assert set(_lib.SIGNATURES) == declared


def test_strerror_version_defaults():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -5, 17):
        assert isinstance(L.dgf_strerror(code), bytes) and len(L.dgf_strerror(code)) > 0
    assert L.dgf_version() >= 100
    o = _lib.DgfTrackOpts()
    assert L.dgf_track_opts_default(ctypes.byref(o)) == 0
    assert (o.sigma1, o.sigma2) == (8.0, 32.0)
    assert abs(o.eps_coarse - 1e-2) < 1e-9 and abs(o.eps_fine - 1e-4) < 1e-10
    assert abs(o.min_eig - 6.5025) < 1e-4 and o.flags == 0 and o.cross_tau == 25.0
    assert L.dgf_track_opts_default(None) == -1


@pytest.mark.parametrize("W,H,w,d,n", [(256, 128, 9, 8, 465), (1242, 375, 9, 5, 18278), (1242, 375, 3, 9, 5796),
                                       (2048, 1024, 9, 2, 518160), (8, 8, 9, 1, 0), (9, 9, 9, 4, 1)])
def test_detect_count(W, H, w, d, n):
    assert _lib.lib().dgf_detect_count(W, H, w, d) == n
    assert _lib.lib().dgf_detect_count(W, H, 0, d) == -1


def test_pyramid_layout_and_workspace():
    L = _lib.lib()
    off = (ctypes.c_int64 * 12)()
    pit = (ctypes.c_int64 * 12)()
    total = L.dgf_pyramid_layout(1242, 375, 5, 0, off, pit)
    dims = [(621, 188), (311, 94), (156, 47), (78, 24)]
    for l, (w, h) in enumerate(dims, start=1):
        assert pit[l] >= w and pit[l] % 64 == 0 and off[l] % 256 == 0
        if l > 1:
            assert off[l] >= off[l - 1] + pit[l - 1] * dims[l - 2][1]
    assert total >= off[4] + pit[4] * 24
    assert L.dgf_pyramid_layout(1242, 375, 1, 0, None, None) == 0
    assert L.dgf_pyramid_layout(1242, 375, 13, 0, None, None) == 0
    assert L.dgf_pyramid_layout(0, 375, 3, 0, None, None) == 0
    f32 = L.dgf_pyramid_layout(1242, 375, 5, 1, None, None)
    assert f32 >= 4 * 621 * 188
    assert L.dgf_track_workspace_bytes(1242, 375, 5, 0) >= 2 * total
    assert L.dgf_track_workspace_bytes(1242, 375, 5, 7) == 0


def _img(data=1 << 20, w=64, h=48, pitch=64, dtype=0):
    return _lib.DgfImage(data, w, h, pitch, dtype)


def test_argument_validation_before_launch():
    """Every one of these is rejected on the host; nothing is launched (no GPU here)."""
    L = _lib.lib()
    bad = [_img(data=0), _img(w=0), _img(pitch=10), _img(dtype=5), _img(dtype=1, pitch=100)]
    for im in bad:
        assert L.dgf_detect(ctypes.byref(im), 9, 8, ctypes.c_void_p(1 << 20), None, None, 100, None) == -1
    im = _img()
    assert L.dgf_detect(None, 9, 8, ctypes.c_void_p(1 << 20), None, None, 100, None) == -1
    assert L.dgf_detect(ctypes.byref(_img(dtype=1, pitch=256)), 9, 8, ctypes.c_void_p(1 << 20), None, None, 100,
                        None) == -1
    assert L.dgf_detect(ctypes.byref(im), 9, 0, ctypes.c_void_p(1 << 20), None, None, 100, None) == -1
    assert L.dgf_detect(ctypes.byref(im), 129, 8, ctypes.c_void_p(1 << 20), None, None, 100, None) == -1
    assert L.dgf_detect(ctypes.byref(im), 9, 8, ctypes.c_void_p(1 << 20), None, None, 3, None) == -2
    assert L.dgf_detect(ctypes.byref(im), 9, 8, None, None, None, 100, None) == -1
    # kernels use 24-bit row x pitch products and 32-bit byte offsets: larger images are rejected
    assert L.dgf_detect(ctypes.byref(_img(pitch=1 << 24)), 9, 8, ctypes.c_void_p(1 << 20), None, None, 100, None) == -1
    assert L.dgf_detect(ctypes.byref(_img(h=1 << 16, pitch=1 << 15)), 9, 8, ctypes.c_void_p(1 << 20), None, None, 100,
                        None) == -1
    # image smaller than the window: nothing to do, nothing launched
    assert L.dgf_detect(ctypes.byref(_img(w=5, h=5, pitch=5)), 9, 8, None, None, None, 0, None) == 0

    P = ctypes.c_void_p(1 << 20)
    ws = L.dgf_track_workspace_bytes(64, 48, 3, 0)

    def track(I0=im, I1=im, pts=P, n=10, levels=3, s=9, iters=10, opts=None, wsp=P, wsb=ws, flow=P, st=P):
        return L.dgf_track(ctypes.byref(I0), ctypes.byref(I1), pts, n, levels, s, iters, opts, wsp, wsb, flow, st, None,
                           None, None)

    assert track(I1=_img(w=63)) == -1
    assert track(I1=_img(dtype=1, pitch=256)) == -1
    assert track(levels=0) == -1 and track(levels=13) == -1
    assert track(s=8) == -1 and track(s=33) == -1 and track(s=0) == -1
    assert track(iters=0) == -1
    assert track(n=-1) == -1
    assert track(pts=None) == -1 and track(flow=None) == -1 and track(st=None) == -1
    assert track(wsp=None) == -5 and track(wsb=ws - 1) == -5
    o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, 8)  # unknown flag
    assert track(opts=ctypes.pointer(o)) == -3
    for fl in (_lib.DGF_TRACK_ILLUM, _lib.DGF_TRACK_CROSS, _lib.DGF_TRACK_GLOBAL):  # no row-run kernel for 13x13
        o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, fl, 25.0)
        assert track(s=13, opts=ctypes.pointer(o)) == -3
    for tau in (float("nan"), -1.0, float("inf")):  # cross-based supports need a finite threshold >= 0
        o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, _lib.DGF_TRACK_CROSS, tau)
        assert track(opts=ctypes.pointer(o)) == -1
    o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, 0, float("nan"))  # the threshold is unused without the flag
    assert track(n=0, pts=None, flow=None, st=None, opts=ctypes.pointer(o)) == 0
    # the global prior keeps its fit in the workspace, so it needs one even for a single level
    o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, _lib.DGF_TRACK_GLOBAL, 25.0)
    assert track(levels=1, wsp=None, wsb=0, opts=ctypes.pointer(o)) == -5
    assert track(levels=1, wsp=None, wsb=0, n=0, pts=None, flow=None, st=None) == 0
    assert track(levels=1, wsp=None, wsb=0, n=0, pts=None, flow=None, st=None, opts=ctypes.pointer(o)) == -5
    o = _lib.DgfTrackOpts(float("nan"), 32, 1e-2, 1e-4, 6.5, 0)
    assert track(opts=ctypes.pointer(o)) == -1
    # n = 0 validates and launches nothing
    assert track(n=0, pts=None, flow=None, st=None) == 0
    assert L.dgf_pyramid(ctypes.byref(im), 3, None, 0, None) == -5
    assert L.dgf_pyramid(ctypes.byref(im), 1, None, 0, None) == 0
    assert L.dgf_track_pyramids(ctypes.byref(im), ctypes.byref(_img(h=47)), 3, P, ws, None) == -1
    assert L.dgf_track_pyramids(ctypes.byref(im), ctypes.byref(im), 3, P, ws - 1, None) == -5


def test_detect_pyramids_argument_checks_before_launch():
    """dgf_detect_pyramids: every rejection happens on the host, before any launch."""
    L = _lib.lib()
    P = ctypes.c_void_p(1 << 20)
    im = _img()
    ws = L.dgf_track_workspace_bytes(64, 48, 3, 0)
    n = L.dgf_detect_count(64, 48, 9, 8)
    assert n == 35

    def run(I0=im, I1=im, window=9, stride=8, levels=3, wsp=P, wsb=ws, pts=P, cap=n):
        return L.dgf_detect_pyramids(ctypes.byref(I0), ctypes.byref(I1), window, stride, levels, wsp, wsb, pts, None,
                                     None, cap, None)

    f32 = _img(dtype=1, pitch=256)
    assert run(I0=f32, I1=f32) == -1 and run(I1=f32) == -1 and run(I1=_img(w=63)) == -1
    assert run(window=0) == -1 and run(window=129) == -1 and run(stride=0) == -1
    assert run(levels=0) == -1 and run(levels=13) == -1
    assert run(pts=None) == -1
    assert run(cap=n - 1) == -2
    assert run(wsp=None) == -5 and run(wsb=ws - 1) == -5


def test_tuning_table_host_only():
    L = _lib.lib()
    t = _lib.DgfTuning()
    assert L.dgf_get_tuning(21, 5, 0, 18278, ctypes.byref(t)) == 0
    assert t.lanes_per_point in (16, 32, 64) and t.waves_per_group in (1, 2, 4) and t.kernel in (0, 1)
    assert L.dgf_get_tuning(8, 5, 0, 10, ctypes.byref(t)) == -1
    assert L.dgf_get_tuning(21, 5, 3, 10, ctypes.byref(t)) == -1
    # install / read back / reject shapes without a kernel
    new = _lib.DgfTuning(32, 2, 3, 1, -1.0)
    assert L.dgf_set_tuning(13, 0, ctypes.byref(new)) == 0
    assert L.dgf_get_tuning(13, 3, 0, 100, ctypes.byref(t)) == 0
    assert (t.lanes_per_point, t.waves_per_group, t.margin, t.kernel) == (32, 2, 3, 1)
    assert L.dgf_set_tuning(31, 0, ctypes.byref(_lib.DgfTuning(16, 1, 2, 1, -1.0))) == -3  # 61 slots: none compiled
    assert L.dgf_set_tuning(13, 0, ctypes.byref(_lib.DgfTuning(24, 1, 2, 1, -1.0))) == -3
    assert L.dgf_set_tuning(13, 0, None) == -1


def test_epic_argument_checks_before_any_launch():
    # every case is rejected on the host, so nothing reaches a device
    import ctypes
    from paper_1901_09971_amd._lib import DgfEpicOpts, DgfImage, lib
    L = lib()
    o = DgfEpicOpts()
    assert L.dgf_epic_opts_default(ctypes.byref(o)) == 0 and (o.k, o.kappa, o.half_dist) == (128, 8, 64)
    P = ctypes.c_void_p(1 << 20)
    W, H, n = 64, 48, 10
    ws = L.dgf_epic_workspace_bytes(W, H, n)
    assert ws >= W * H * 10

    def call(img=None, k=128, kappa=8, hd=64, n=n, wsb=ws, pitch=2 * W, dense=P, nbr=None, nbr_dist=None):
        im = img or DgfImage(1 << 20, W, H, W, 0)
        oo = DgfEpicOpts(k, kappa, hd)
        return L.dgf_epic(ctypes.byref(im), P, P, P, n, ctypes.byref(oo), P, wsb, dense, pitch, None, None, nbr,
                          nbr_dist, None, None)

    assert call(img=DgfImage(1 << 20, W, H, 4 * W, 1)) == -1  # float frame
    assert call(k=0) == -1 and call(k=257) == -1 and call(kappa=0) == -1 and call(hd=0) == -1
    assert call(n=-1) == -1
    assert call(pitch=2 * W - 2) == -1 and call(pitch=2 * W + 1) == -1 and call(dense=None) == -1
    assert call(nbr=P) == -1  # nbr and nbr_dist go together
    assert call(wsb=ws - 1) == -5
    # distances must fit 32 bits: (W + H - 2) (kappa + 1020) <= 2^32 - 2
    assert call(img=DgfImage(1 << 20, 8000, 10, 8000, 0), kappa=1 << 20) == -3

    # the form without host synchronisation: the same checks, and a status word and a launch count
    def call_async(max_relax=0, status_out=P, **kw):
        im = DgfImage(1 << 20, W, H, W, 0)
        oo = DgfEpicOpts(128, 8, 64)
        return L.dgf_epic_async(ctypes.byref(im), P, P, P, kw.get("n", n), ctypes.byref(oo), P, kw.get("wsb", ws),
                                P, 2 * W, None, None, None, None, None, max_relax, status_out, None)

    assert call_async(status_out=None) == -1 and call_async(status_out=ctypes.c_void_p((1 << 20) + 2)) == -1
    assert call_async(max_relax=-1) == -1 and call_async(max_relax=(1 << 14) + 1) == -1
    assert call_async(n=-1) == -1 and call_async(wsb=ws - 1) == -5


def test_track_static_checks_before_any_hip_call():
    """dgf_track_static rejects bad arguments and inputs larger than its static scratch on the
    host, before it looks up the scratch array or launches anything (no GPU here)."""
    L = _lib.lib()
    P = ctypes.c_void_p(1 << 20)
    im = _img()

    def call(I0=im, I1=im, pts=P, n=10, levels=3, s=9, iters=10, opts=None, flow=P, st=P, ill=None):
        return L.dgf_track_static(ctypes.byref(I0), ctypes.byref(I1), pts, n, levels, s, iters, opts, flow, st, None,
                                  ill, None)

    assert call(I1=_img(w=63)) == -1 and call(levels=0) == -1 and call(levels=13) == -1
    assert call(s=8) == -1 and call(iters=0) == -1 and call(n=-1) == -1
    assert call(pts=None) == -1 and call(flow=None) == -1 and call(st=None) == -1
    assert call(ill=P) == -1  # illum_out without the illumination model
    o = _lib.DgfTrackOpts(8, 32, 1e-2, 1e-4, 6.5, 8)
    assert call(opts=ctypes.pointer(o)) == -3
    assert L.dgf_track_static(None, ctypes.byref(im), P, 10, 3, 9, 10, None, P, P, None, None, None) == -1
    # n = 0: validated, nothing looked up or launched
    assert call(n=0, pts=None, flow=None, st=None) == 0
    # pyramids larger than the static array: DGF_ERR_SCRATCH, whatever the point count
    big = _img(w=4096, h=4096, pitch=4 * 4096, dtype=1)
    need = L.dgf_track_workspace_bytes(4096, 4096, 3, 1)
    assert need > _lib.DGF_TRACK_STATIC_MAX_BYTES
    assert call(I0=big, I1=big) == _lib.DGF_ERR_SCRATCH
    assert call(I0=big, I1=big, n=0, pts=None, flow=None, st=None) == _lib.DGF_ERR_SCRATCH
    # one level needs no pyramid: never too large
    assert L.dgf_track_workspace_bytes(4096, 4096, 1, 1) <= _lib.DGF_TRACK_STATIC_MAX_BYTES
    assert b"static scratch" in L.dgf_strerror(_lib.DGF_ERR_SCRATCH)
