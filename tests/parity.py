"""Tracking parity between the GPU and the FP64 oracle on the same float32 points, class by class.

* CONVERGED on both sides: the level-0 flow solves the robust fixed-point equation on both sides;
  FP32 against FP64 must agree within ``tol`` (1e-3 px).
* ILL_CONDITIONED on both sides: the flow is the guess propagated from the coarser levels,
  u = 2 (g_1 + d_1).  The coarser levels stop on |step| < eps_coarse, so two evaluations that stop
  one iteration apart differ by up to about 2^l eps_coarse, and a coarse level that ran out of
  iterations hands on an iterate, not a solution.  Where both sides ran the same number of
  iterations and every coarse level stopped on the step test (the oracle's per-level counts are
  below the limit), the guess is the same computation and must agree within ``tol`` (``ill_tol``
  where given: a coarse level that converges slowly stops at an iterate whose distance from its
  fixed point is several times eps_coarse, and the rounding of either side moves that stopping
  point by a part of it).  The other points are counted and reported.
* NOT_CONVERGED on both sides: level 0 ran out of iterations, so the flow is an iterate, not a
  solution; its difference is reported as a distribution, and where there are at least 20 such
  points (enough for a median) the median is held to ``nc_median``.
* Status agreement over all points must reach ``min_agree``.
* ``paths="determined"`` (used with small adaptive supports): a coarse level that runs out of
  iterations hands on an iterate, not a solution, and where the supports are small that iterate
  depends chaotically on rounding, so the finer levels can settle on a different solution on each
  side.  Then the CONVERGED bound and ``min_agree`` apply to the points whose coarse levels all
  stopped on the step test in the oracle (a determined path); the others are counted and reported,
  and agreement over all points must still reach ``min_agree_all``.
"""
import numpy as np

ST_CONV, ST_NC, ST_ILL, ST_OOB = 0, 1, 2, 3


def compare_tracks(g_flow, g_st, o_flow, o_st, min_agree, tol=1e-3, g_its=None, o_its=None, iters=None,
                   nc_median=1e-3, label="", paths="all", min_agree_all=0.99, ill_tol=None):
    g_flow = np.asarray(g_flow, np.float64)
    o_flow = np.asarray(o_flow, np.float64)
    n = len(g_st)
    # coarse levels that all stopped on the step test in the oracle (per-level counts, coarsest first)
    determined = np.ones(n, bool)
    if o_its is not None and iters is not None:
        determined = np.all(np.asarray(o_its).reshape(n, -1)[:, :-1] < iters, axis=1)
    held = determined if paths == "determined" else np.ones(n, bool)
    agree_all = float(np.mean(g_st == o_st)) if n else 1.0
    agree = float(np.mean(g_st[held] == o_st[held])) if held.any() else 1.0
    conv_all = (g_st == ST_CONV) & (o_st == ST_CONV)
    conv = conv_all & held
    err_conv = float(np.abs(g_flow[conv] - o_flow[conv]).max()) if conv.any() else 0.0
    n_free = int((conv_all & ~held).sum())
    err_free = float(np.abs(g_flow[conv_all & ~held] - o_flow[conv_all & ~held]).max()) if n_free else 0.0
    ill = (g_st == ST_ILL) & (o_st == ST_ILL)
    same = ill & determined
    if g_its is not None and o_its is not None:
        o_lv = np.asarray(o_its).reshape(n, -1)
        same &= np.asarray(g_its) == o_lv.sum(1)
    d_ill = np.abs(g_flow[same] - o_flow[same]).max(1) if same.any() else np.zeros(0)
    err_ill = float(d_ill.max()) if len(d_ill) else 0.0
    nc = (g_st == ST_NC) & (o_st == ST_NC) & np.all(np.isfinite(g_flow), 1) & np.all(np.isfinite(o_flow), 1)
    d_nc = np.linalg.norm(g_flow[nc] - o_flow[nc], axis=1) if nc.any() else np.zeros(0)
    q = np.percentile(d_nc, [50, 90, 99]) if len(d_nc) else np.zeros(3)
    if paths == "determined":
        print(f"{label} determined paths {int(determined.sum())}/{n}, agree over all {agree_all:.5f}; "
              f"converged on undetermined paths {n_free}, max_err {err_free:.2e}", flush=True)
    print(f"{label} n={n} agree={agree:.5f} conv={int(conv.sum())} max_err={err_conv:.2e} "
          f"ill={int(ill.sum())} (same path {int(same.sum())}, max_err {err_ill:.2e}) "
          f"not_conv={int(nc.sum())} |dflow| p50/p90/p99 {q[0]:.2e}/{q[1]:.2e}/{q[2]:.2e} "
          f"gpu_st={np.bincount(g_st, minlength=4)} orc_st={np.bincount(o_st, minlength=4)}", flush=True)
    assert err_conv <= tol, (label, err_conv)
    assert err_ill <= (tol if ill_tol is None else ill_tol), (label, err_ill)
    assert agree >= min_agree, (label, agree)
    if paths == "determined":
        assert agree_all >= min_agree_all, (label, agree_all)
    if nc_median is not None and len(d_nc) >= 20:
        assert q[0] <= nc_median, (label, q[0])
    return dict(agree=agree, conv=int(conv.sum()), err_conv=err_conv, ill_same=int(same.sum()), err_ill=err_ill,
                nc=int(nc.sum()), nc_q=q)
