"""Pins of the FP64 oracle of the dense interpolation (Section 2 "Interpolation": an affine motion
fitted to the k nearest tracked points under a geodesic distance over an image-gradient edge
map; k = 128 in Section 3).  Each check holds by construction of the method, not by re-running
the oracle's own code: closed forms, brute force with scipy's graph routines on small inputs,
exact recovery of affine motion, and the edge-preserving property itself."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra

import oracle


def _grid_graph(E, kappa):
    """4-connected pixel graph with step cost kappa + E(p) + E(q), built independently."""
    H, W = E.shape
    idx = np.arange(H * W).reshape(H, W)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    Ef = E.ravel().astype(np.float64)
    w = kappa + Ef[a] + Ef[b]
    return coo_matrix((np.concatenate([w, w]), (np.concatenate([a, b]), np.concatenate([b, a]))),
                      shape=(H * W, H * W)).tocsr()


def _seed_pixels(pts, W, H):
    px = np.clip(np.floor(pts[:, 0] + 0.5).astype(int), 0, W - 1)
    py = np.clip(np.floor(pts[:, 1] + 0.5).astype(int), 0, H - 1)
    return py * W + px


def _brute_voronoi(I, pts, status, kappa):
    H, W = I.shape
    E = oracle.epic_edges(I)
    G = _grid_graph(E, kappa)
    sp = _seed_pixels(pts, W, H)
    alive = np.zeros(len(pts), bool)
    taken = set()
    for i in range(len(pts)):
        if status[i] == 0 and sp[i] not in taken:
            alive[i] = True
            taken.add(sp[i])
    ids = np.nonzero(alive)[0]
    dist = dijkstra(G, indices=sp[ids])  # [n_alive, H*W]
    D = dist.min(axis=0)
    # lowest index among the seeds at the least distance (ids are increasing)
    L = ids[np.argmax(dist == D[None, :], axis=0)]
    return D.reshape(H, W), L.reshape(H, W), alive


def test_edges_closed_form():
    x = np.arange(12)[None, :]
    y = np.arange(9)[:, None]
    I = (3 * x + 7 * y).astype(np.uint8)  # at most 33 + 56
    E = oracle.epic_edges(I)
    # interior: |2a| + |2b|; a border column or row sees a one-sided difference |a| or |b|
    assert np.all(E[1:-1, 1:-1] == 2 * 3 + 2 * 7)
    assert np.all(E[1:-1, 0] == 3 + 14) and np.all(E[1:-1, -1] == 3 + 14)
    assert np.all(E[0, 1:-1] == 6 + 7) and np.all(E[-1, 1:-1] == 6 + 7)
    assert E[0, 0] == 3 + 7
    # a vertical step of height 200 between columns 5 and 6
    S = np.zeros((6, 12), np.uint8)
    S[:, 6:] = 200
    Es = oracle.epic_edges(S)
    assert np.all(Es[:, 5] == 200) and np.all(Es[:, 6] == 200)
    assert np.all(Es[:, :5] == 0) and np.all(Es[:, 7:] == 0)


def test_voronoi_flat_image_is_manhattan():
    W, H, kappa = 23, 17, 5
    I = np.full((H, W), 90, np.uint8)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.uniform(0, W - 1, 9), rng.uniform(0, H - 1, 9)], 1)
    st = np.zeros(9, np.uint8)
    D, L, alive = oracle.epic_voronoi(I, pts, st, kappa)
    sp = _seed_pixels(pts, W, H)
    sx, sy = sp % W, sp // W
    yy, xx = np.mgrid[0:H, 0:W]
    man = np.abs(xx[None] - sx[:, None, None]) + np.abs(yy[None] - sy[:, None, None])
    live = np.nonzero(alive)[0]
    dmin = man[live].min(axis=0)
    assert np.array_equal(D, kappa * dmin)
    Lb = live[np.argmax(man[live] == dmin[None], axis=0)]
    assert np.array_equal(L, Lb)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_voronoi_brute_force_on_random_images(seed):
    rng = np.random.default_rng(seed)
    W, H = 26, 19
    I = rng.integers(0, 256, (H, W)).astype(np.uint8)
    I[:, 13:] //= 3  # an edge
    n = 12
    pts = np.stack([rng.uniform(-0.4, W - 0.6, n), rng.uniform(-0.4, H - 0.6, n)], 1)
    pts[5] = np.floor(pts[2] + 0.5) + [0.3, -0.2]  # same seed pixel as a lower index: dropped
    st = np.zeros(n, np.uint8)
    st[7] = 1  # not converged: not a seed
    D, L, alive = oracle.epic_voronoi(I, pts, st, 3)
    Db, Lb, ab = _brute_voronoi(I, pts, st, 3)
    assert np.array_equal(alive.astype(bool), ab)
    assert not alive[5] and not alive[7]
    assert np.array_equal(D, Db.astype(np.int64))
    assert np.array_equal(L, Lb)


def _brute_neighbours(I, D, L, alive, kappa, k, h):
    """Seed graph from (D, L) and Dijkstra on it with scipy; the k nearest by (distance, index)
    within 64 h."""
    H, W = I.shape
    E = oracle.epic_edges(I).astype(np.int64)
    n = len(alive)
    best = {}
    for (dy, dx) in ((0, 1), (1, 0)):
        a = (slice(0, H - dy), slice(0, W - dx))
        b = (slice(dy, H), slice(dx, W))
        s, t = L[a].ravel(), L[b].ravel()
        w = (D[a] + kappa + E[a] + E[b] + D[b]).ravel()
        for si, ti, wi in zip(s, t, w):
            if si == ti:
                continue
            for key in ((si, ti), (ti, si)):
                if key not in best or wi < best[key]:
                    best[key] = wi
    rows = np.array([k_[0] for k_ in best], int)
    cols = np.array([k_[1] for k_ in best], int)
    vals = np.array([best[k_] for k_ in best], np.float64)
    G = coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    dist = dijkstra(G, indices=np.nonzero(alive)[0])
    out_nb, out_nd = {}, {}
    for r, s in enumerate(np.nonzero(alive)[0]):
        d = dist[r]
        cand = [(int(d[t]), t) for t in range(n) if np.isfinite(d[t]) and d[t] <= 64 * h]
        cand.sort()
        out_nb[s] = [t for _, t in cand[:k]]
        out_nd[s] = [dd for dd, _ in cand[:k]]
    return out_nb, out_nd


@pytest.mark.parametrize("k", [4, 7, 128])
def test_neighbours_brute_force(k):
    rng = np.random.default_rng(11)
    W, H = 40, 30
    I = (rng.integers(0, 40, (H, W)) + np.where(np.arange(W)[None, :] > 21, 150, 0)).astype(np.uint8)
    n = 30
    pts = np.stack([rng.uniform(0, W - 1, n), rng.uniform(0, H - 1, n)], 1)
    fl = rng.normal(size=(n, 2))
    st = np.zeros(n, np.uint8)
    kappa, h = 4, 20
    _, aux = oracle.epic(I, pts, fl, st, k=k, kappa=kappa, h=h, full=True)
    nb_b, nd_b = _brute_neighbours(I, aux["D"], aux["L"], aux["alive"], kappa, k, h)
    for s in np.nonzero(aux["alive"])[0]:
        cnt = len(nb_b[s])
        assert list(aux["nb"][s, :cnt]) == nb_b[s]
        assert list(aux["nd"][s, :cnt]) == nd_b[s]
        assert np.all(aux["nb"][s, cnt:] == -1)
    # the 64 h cut-off binds for some seeds at this h
    if k == 128:
        assert (aux["nb"][aux["alive"] == 1] == -1).any()


def test_fit_is_weighted_least_squares():
    rng = np.random.default_rng(5)
    W, H = 60, 44
    I = rng.integers(0, 60, (H, W)).astype(np.uint8)
    n = 40
    pts = np.stack([rng.uniform(0, W - 1, n), rng.uniform(0, H - 1, n)], 1)
    fl = rng.normal(size=(n, 2)) * 3
    st = np.zeros(n, np.uint8)
    k, kappa, h = 16, 8, 64
    dense, aux = oracle.epic(I, pts, fl, st, k=k, kappa=kappa, h=h, full=True)
    for s in np.nonzero(aux["alive"])[0]:
        m = aux["nb"][s] >= 0
        nb, nd = aux["nb"][s][m], aux["nd"][s][m]
        w = 2.0 ** (-nd / h)
        X = np.stack([pts[nb, 0] - pts[s, 0], pts[nb, 1] - pts[s, 1], np.ones(len(nb))], 1)
        sw = np.sqrt(w)[:, None]
        sol = np.linalg.lstsq(X * sw, fl[nb] * sw, rcond=None)[0]  # [3, 2]
        assert np.allclose(aux["model"][s, :3], sol[:, 0], atol=1e-9)
        assert np.allclose(aux["model"][s, 3:], sol[:, 1], atol=1e-9)
    # every pixel takes its cell's model at its own coordinates
    yy, xx = np.mgrid[0:H, 0:W]
    L = aux["L"]
    M = aux["model"][L]
    rx, ry = xx - pts[L, 0], yy - pts[L, 1]
    assert np.allclose(dense[..., 0], M[..., 0] * rx + M[..., 1] * ry + M[..., 2], atol=1e-12)
    assert np.allclose(dense[..., 1], M[..., 3] * rx + M[..., 4] * ry + M[..., 5], atol=1e-12)


def test_fit_with_weights_spanning_many_binades():
    # h = 1 with a unit step cost: neighbour weights fall to 2^-50 within a few pixels; the fit
    # is still the weighted least-squares minimiser (numpy's SVD solver, ~cond * eps)
    rng = np.random.default_rng(3)
    W, H = 150, 90
    I0 = (rng.integers(0, 30, (H, W)) + np.where(np.arange(W)[None, :] > 70, 120, 0)).astype(np.uint8)
    n = 700
    pts = np.stack([rng.uniform(0, W - 1, n), rng.uniform(0, H - 1, n)], 1)
    fl = rng.normal(size=(n, 2))
    st = np.zeros(n, np.uint8)
    _, aux = oracle.epic(I0, pts, fl, st, k=3, kappa=1, h=1, full=True)
    worst_cond = 0.0
    for s in np.nonzero(aux["alive"])[0]:
        m = aux["nb"][s] >= 0
        nb, nd = aux["nb"][s][m], aux["nd"][s][m]
        if np.all(aux["model"][s, [0, 1, 3, 4]] == 0):
            continue  # weighted mean
        sw = np.sqrt(2.0 ** (-nd / 1.0))[:, None]
        X = np.stack([pts[nb, 0] - pts[s, 0], pts[nb, 1] - pts[s, 1], np.ones(len(nb))], 1) * sw
        worst_cond = max(worst_cond, np.linalg.cond(X))
        sol = np.linalg.lstsq(X, fl[nb] * sw, rcond=None)[0]
        ref = np.concatenate([sol[:, 0], sol[:, 1]])
        assert np.abs(aux["model"][s] - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max()), s
    assert worst_cond > 1e7


def test_affine_motion_is_reproduced_exactly():
    # (a low-contrast texture, so that every seed has enough neighbours for a full affine fit)
    rng = np.random.default_rng(7)
    W, H = 80, 50
    I = rng.integers(0, 12, (H, W)).astype(np.uint8)
    n = 120
    pts = np.stack([rng.uniform(0, W - 1, n), rng.uniform(0, H - 1, n)], 1)
    A = np.array([[0.02, -0.05], [0.03, 0.01]])
    b = np.array([4.0, -2.5])
    fl = pts @ A.T + b
    st = np.zeros(n, np.uint8)
    dense, aux = oracle.epic(I, pts, fl, st, full=True)
    assert np.all(aux["model"][:, [0, 1, 3, 4]] != 0)  # no seed fell back to the mean
    yy, xx = np.mgrid[0:H, 0:W]
    ref = np.stack([xx, yy], -1) @ A.T + b
    assert np.abs(dense - ref).max() < 1e-9


def test_collinear_seeds_take_the_weighted_mean():
    W, H = 30, 20
    I = np.full((H, W), 10, np.uint8)
    pts = np.array([[3.0, 10.0], [9.0, 10.0], [15.0, 10.0], [24.0, 10.0]])
    fl = np.array([[1.0, 0.0], [2.0, 1.0], [4.0, -1.0], [0.5, 3.0]])
    st = np.zeros(4, np.uint8)
    dense, aux = oracle.epic(I, pts, fl, st, k=3, kappa=8, h=64, full=True)
    for s in range(4):
        nb, nd = aux["nb"][s], aux["nd"][s]
        w = 2.0 ** (-nd / 64.0)
        mean = (w[:, None] * fl[nb]).sum(0) / w.sum()
        assert np.allclose(aux["model"][s], [0, 0, mean[0], 0, 0, mean[1]], atol=1e-12)
    # two seeds only: always the mean
    dense2, aux2 = oracle.epic(I, pts[:2], fl[:2], st[:2], full=True)
    assert np.all(aux2["model"][:, [0, 1, 3, 4]] == 0)


def test_non_finite_points_are_not_seeds():
    I = np.full((10, 12), 50, np.uint8)
    pts = np.array([[np.nan, 3.0], [4.0, 4.0], [7.0, 2.0]])
    fl = np.array([[1.0, 1.0], [2.0, -1.0], [np.inf, 0.0]])
    dense, aux = oracle.epic(I, pts, fl, np.zeros(3, np.uint8), full=True)
    assert list(aux["alive"]) == [0, 1, 0]
    assert np.all(dense[..., 0] == 2.0) and np.all(dense[..., 1] == -1.0)


def test_single_seed_and_no_seed():
    I = np.random.default_rng(0).integers(0, 256, (12, 15)).astype(np.uint8)
    pts = np.array([[4.2, 6.7], [8.0, 3.0]])
    fl = np.array([[1.5, -2.0], [9.0, 9.0]])
    dense = oracle.epic(I, pts, fl, np.array([0, 2], np.uint8))
    assert np.all(dense[..., 0] == 1.5) and np.all(dense[..., 1] == -2.0)
    dense0 = oracle.epic(I, pts, fl, np.array([1, 2], np.uint8))
    assert np.all(np.isnan(dense0))


def test_edges_keep_motions_apart():
    # two flat regions with opposite motions, seeds on a grid in both; with the step edge the
    # geodesic neighbours of a point stay on its side, on a flat image they do not
    W, H = 96, 64
    I = np.full((H, W), 40, np.uint8)
    I[:, 48:] = 220
    gx, gy = np.meshgrid(np.arange(2.0, W, 5.0), np.arange(2.0, H, 5.0))
    pts = np.stack([gx.ravel(), gy.ravel()], 1)
    fl = np.where(pts[:, :1] < 47.5, [[5.0, 0.0]], [[-5.0, 1.0]])
    st = np.zeros(len(pts), np.uint8)
    dense = oracle.epic(I, pts, fl, st)
    xx = np.arange(W)
    left, right = xx <= 44, xx >= 51
    assert np.abs(dense[:, left] - [5.0, 0.0]).max() < 0.05
    assert np.abs(dense[:, right] - [-5.0, 1.0]).max() < 0.05
    flat = oracle.epic(np.full((H, W), 40, np.uint8), pts, fl, st)
    assert np.abs(flat[:, left] - [5.0, 0.0]).max() > 1.0


def test_flow_error_by_hand():
    f = np.array([[[0.0, 0.0], [3.0, 4.0]], [[1.0, 1.0], [0.0, 2.0]]])
    r = np.zeros_like(f)
    valid = np.array([[1, 1], [0, 1]], np.uint8)
    epe, out, cnt = oracle.flow_error(f, r, valid, 3.0)
    assert cnt == 3 and abs(epe - (0 + 5 + 2) / 3) < 1e-15 and abs(out - 1 / 3) < 1e-15
