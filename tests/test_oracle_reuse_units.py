"""Crafted-input pins of the oracle's reuse passes (closed forms and
distributions that an unbiasedness test cannot see).

* luminance reading: in the white furnace every RIS weight equals
  lum(rho * L) with Rec. 709 weights, so wsum = M * lum(rho * L);
* view-path bias: the query point lies on the segment [y, x] at distance
  min(d, |x - y| / 2) from y, and for real path vertices it is never inside
  geometry (Sec. 3.4);
* temporal history cap: M_out = M + min(M_hist, m_cap * M);
* temporal normalisation uses the previous frame's vertex for the history
  domain: if that vertex cannot see y, only the current domain counts and
  W = W_hist * M_hist / M;
* spatial weighted-reservoir selection: with identical samples, a neighbour
  is chosen with probability W_q M_q / sum W M, and the merged W is the
  M-weighted mean of the W_q (all domains see the sample).
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as o
from paper_2108_05263_amd import scenegen as g


def test_luminance_reading_in_furnace():
    rho = np.array([0.5, 0.7, 0.9], np.float32)
    L = np.array([1.0, 2.0, 3.0], np.float32)
    sc = g.furnace_plane(albedo=rho, sky=L)
    cam = g.furnace_camera(16, 12)
    grid = g.probe_grid((2, 2, 2), (-1, -1, -1), 1.0)
    irr, dep = g.empty_probe_textures(grid)
    pr = g.Params(M=6, k=3, n_spatial=0, radius=3.0, temporal=False)
    gb = o.gbuffer(sc, cam)
    res, _ = o.resample_initial(sc, 16, 12, gb, grid, irr, dep, pr, 4, 0)
    on = gb[:, 13] != o.MISS
    rl = rho.astype(np.float64) * L.astype(np.float64)
    lum709 = 0.2126 * rl[0] + 0.7152 * rl[1] + 0.0722 * rl[2]
    assert np.allclose(res[on, 9], pr.M * lum709, rtol=1e-13)


def _sdf(scene, p):
    rec = scene.prims
    types = rec.view(np.uint32)[:, 3]
    best = np.full(p.shape[0], np.inf)
    for i in range(len(rec)):
        c, s = rec[i, 0:3].astype(np.float64), rec[i, 4:7].astype(np.float64)
        if types[i] == 0:
            d = np.linalg.norm(p - c, axis=1) - s[0]
        else:
            q = np.abs(p - c) - s
            d = np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)
        best = np.minimum(best, d)
    lo, hi = scene.room_lo.astype(np.float64), scene.room_hi.astype(np.float64)
    wall = np.minimum((p - lo).min(axis=1), (hi - p).min(axis=1))
    return np.minimum(best, wall)


def test_view_bias_segment_and_never_inside():
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg, width=24, height=24)
    gb = o.gbuffer(sc, cam)
    rng = np.random.default_rng(3)
    d = 0.6
    pts = []
    for p in rng.choice(np.where(gb[:, 13] != o.MISS)[0], 150, replace=False):
        x, nx = gb[p, 0:3], gb[p, 3:6]
        w = o.cosine_dir(nx, rng.random(), rng.random())
        hit, t, prim, ny = o.closest_hit(sc, x + sc.eps * nx, w)
        y = x + sc.eps * nx + t * w
        pb = o.view_bias(y, x, d)
        dist = np.linalg.norm(x - y)
        # on the segment, at the stated distance from y
        assert np.linalg.norm(pb - y) == pytest.approx(min(d, dist / 2), rel=1e-12)
        assert np.linalg.norm(pb - y) + np.linalg.norm(x - pb) == pytest.approx(dist, rel=1e-12)
        pts.append(pb)
    # never inside a primitive or outside the room
    assert np.all(_sdf(sc, np.array(pts)) > 0.0)


@pytest.mark.parametrize("m_cap", [3.0, 2.3])
def test_temporal_history_cap(m_cap):
    """The history's M is capped at floor(m_cap (M + M_light)), a multiple of
    the per-frame candidate count (a non-integer multiple rounds down)."""
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg, width=16, height=16)
    grid = g.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    pr = g.Params(M=4, k=3, n_spatial=2, radius=3.0, temporal=True, m_cap=m_cap)
    cap = math.floor(m_cap * pr.M)
    seq = o.Sequence(sc, grid, irr, dep, pr, 5)
    hist = None
    for f in range(3):
        img, st = seq.frame(cam, f)
        if f > 0:
            cur, out = st["initial"], st["temporal"]
            active = (st["gbuffer"][:, 13] != o.MISS) & (st["gbuffer"][:, 6:9].max(1) > 0)
            # static camera: every active pixel's history is its own previous reservoir
            expect = cur[:, 11] + np.minimum(hist[:, 11], cap)
            assert np.array_equal(out[active, 11], expect[active])
            assert np.any(hist[active, 11] > cap)
        hist = st["spatial1"]


def test_subsampled_pixels_take_over_their_history():
    """Candidate subsampling (Sec. 6): a pixel that draws no candidates this
    frame has M = 0 after the initial pass, and temporal reuse fills it from
    its history (capped at the per-frame candidate count, not at its own M)."""
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg, width=16, height=16)
    grid = g.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    pr = g.Params(M=4, k=0, n_spatial=0, temporal=True, m_cap=3, subsample=2)
    seq = o.Sequence(sc, grid, irr, dep, pr, 5)
    _, st0 = seq.frame(cam, 0)
    _, st1 = seq.frame(cam, 1)
    gb = st1["gbuffer"]
    active = (gb[:, 13] != o.MISS) & (gb[:, 6:9].max(1) > 0)
    p = np.arange(16 * 16)
    off = active & (((p % 16) + (p // 16) + 1) % 2 != 0)        # drew nothing in frame 1
    on0 = active & (((p % 16) + (p // 16) + 0) % 2 == 0)        # drew in frame 0
    assert off.sum() > 20 and np.array_equal(off, on0 & active)
    assert np.all(st1["initial"][off, 11] == 0)
    hist = st0["temporal"] if "temporal" in st0 else st0["initial"]
    # the history of these pixels (static camera: their own previous reservoir)
    out = st1["temporal"]
    assert np.array_equal(out[off, 11], np.minimum(hist[off, 11], 3 * pr.M))
    assert np.all(out[off, 11] > 0)
    held = off & (hist[:, 10] > 0)
    assert held.sum() > 10
    # the sample is taken over: same tag, and W = wsum / (Z p_hat) > 0 where visible
    assert np.array_equal(out[held, 12], hist[held, 12])
    assert np.mean(out[held, 10] > 0) > 0.9


def _single_pixel_camera(eye, look):
    eye = np.asarray(eye, np.float64)
    f = np.asarray(look, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return g.Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32),
                    right=r.astype(np.float32), up=u.astype(np.float32),
                    tan_half_fovy=float(np.float32(0.5)), width=1, height=1)


def _gb_record(pos, nrm, alb, depth, prim=0):
    r = np.zeros(14)
    r[0:3], r[3:6], r[6:9], r[12], r[13] = pos, nrm, alb, depth, prim
    return r


def test_temporal_history_domain_uses_previous_vertex():
    sc = g.shadow_scene()       # floor top y=0; wall z in [-0.05, 0.05], y in [0, 1]
    x = np.array([0.0, 0.0, 1.5])
    x_prev = np.array([0.0, 0.0, -0.3])      # behind the wall
    y = np.array([0.0, 0.9, 2.5])            # a floor-facing point in front of the wall
    ny = np.array([0.0, -1.0, 0.0])
    up = np.array([0.0, 1.0, 0.0])
    assert o.visible(sc, x, up, y, ny) and not o.visible(sc, x_prev, up, y, ny)
    cam = _single_pixel_camera([0.0, 3.0, 1.5 + 1e-3], x)
    depth = float(np.linalg.norm(cam.eye.astype(np.float64) - x))
    gb = _gb_record(x, up, [0.5, 0.5, 0.5], depth)[None]
    gb_prev = _gb_record(x_prev, up, [0.5, 0.5, 0.5], depth)[None]
    M = 4.0
    cur = np.zeros((1, 14))
    cur[0, 11], cur[0, 12], cur[0, 13] = M, float(0xFFFFFFFF), float(o.MISS)
    hist = np.zeros((1, 14))
    hist[0, 0:3], hist[0, 3:6], hist[0, 6:9] = y, ny, [3.0, 2.0, 1.0]
    Wh, Mh = 0.37, 9.0
    hist[0, 10], hist[0, 11], hist[0, 12], hist[0, 13] = Wh, Mh, 77.0, 0.0
    pr = g.Params(M=4, temporal=True, m_cap=20)
    out = o.resample_temporal(sc, 1, 1, gb, gb_prev, cam, cur, hist, pr, 1, 1)
    assert out[0, 12] == 77.0 and out[0, 11] == M + Mh
    assert out[0, 10] == pytest.approx(Wh * Mh / M, rel=1e-12)
    # control: a history vertex that sees y counts too
    gb_prev2 = _gb_record(x + np.array([0.0, 0.0, 0.01]), up, [0.5] * 3, depth)[None]
    out2 = o.resample_temporal(sc, 1, 1, gb, gb_prev2, cam, cur, hist, pr, 1, 1)
    assert out2[0, 10] == pytest.approx(Wh * Mh / (M + Mh), rel=1e-12)


def test_spatial_selection_frequencies_and_weight():
    sc = g.furnace_plane(albedo=(0.5, 0.5, 0.5), sky=(1.0, 1.0, 1.0))
    W = H = 9
    n = W * H
    gb = np.zeros((n, 14))
    for p in range(n):
        gb[p] = _gb_record([0.01 * (p % W), 0.0, 0.01 * (p // W)], [0, 1.0, 0], [0.5] * 3, 1.0)
    res = np.zeros((n, 14))
    sky_dir = np.array([0.3, 0.9, 0.1])
    sky_dir /= np.linalg.norm(sky_dir)
    Wq = 1.0 + (np.arange(n) % 7)
    Mq = 1.0 + (np.arange(n) % 5)
    res[:, 0:3] = sky_dir
    res[:, 6:9] = 1.0
    res[:, 10], res[:, 11], res[:, 12] = Wq, Mq, np.arange(n)
    res[:, 13] = float(o.MISS)
    pr = g.Params(M=4, k=4, radius=3.0)
    centre = 4 * W + 4
    K = pr.k + 1
    obs, exp_, var = np.zeros(K), np.zeros(K), np.zeros(K)
    for seed in range(3000):
        out = o.resample_spatial(sc, W, H, gb, res, pr, 0, seed, 0, pixels=[centre])
        doms = [centre]
        for j in range(pr.k):
            q = o.spatial_candidate(W, H, centre, j, pr.radius, seed, 0, 0)
            if q >= 0:
                doms.append(q)
        wts = np.array([Wq[d] * Mq[d] for d in doms])
        # merged W: wsum / (Z phat) with identical samples = sum W M / sum M
        assert out[centre, 10] == pytest.approx(wts.sum() / Mq[doms].sum(), rel=1e-12)
        assert out[centre, 11] == Mq[doms].sum()
        pj = wts / wts.sum()
        sel = doms.index(int(out[centre, 12]))
        obs[sel] += 1
        exp_[:len(pj)] += pj
        var[:len(pj)] += pj * (1 - pj)
    # selection frequency at every position of the merge order matches W_q M_q / sum
    z = (obs - exp_) / np.sqrt(var + 1e-12)
    assert np.all(np.abs(z) < 4.5), z


def test_spatial_rejects_dissimilar_neighbours():
    """Neighbours whose view depth differs by more than 10% or whose normal is
    more than 25 degrees away are neither merged nor counted."""
    sc = g.furnace_plane(albedo=(0.5, 0.5, 0.5), sky=(1.0, 1.0, 1.0))
    W = H = 9
    n = W * H
    rng = np.random.default_rng(0)
    cls = rng.integers(0, 4, n)     # 0 ok, 1 depth +20%, 2 normal 30 deg, 3 depth +5% and 20 deg
    gb = np.zeros((n, 14))
    for p in range(n):
        ang = {0: 0.0, 1: 0.0, 2: 30.0, 3: 20.0}[int(cls[p])]
        nrm = [math.sin(math.radians(ang)), math.cos(math.radians(ang)), 0.0]
        depth = {0: 1.0, 1: 1.2, 2: 1.0, 3: 1.05}[int(cls[p])]
        gb[p] = _gb_record([0.01 * (p % W), 0.0, 0.01 * (p // W)], nrm, [0.5] * 3, depth)
    centre = 4 * W + 4
    gb[centre] = _gb_record([0.04, 0.0, 0.04], [0, 1.0, 0], [0.5] * 3, 1.0)
    res = np.zeros((n, 14))
    res[:, 0:3] = [0.0, 1.0, 0.0]
    res[:, 6:9] = 1.0
    res[:, 10], res[:, 11], res[:, 12], res[:, 13] = 1.0, 3.0, np.arange(n), float(o.MISS)
    pr = g.Params(M=4, k=5, radius=4.0)
    seen = set()
    for seed in range(200):
        out = o.resample_spatial(sc, W, H, gb, res, pr, 0, seed, 0, pixels=[centre])
        merged = 1
        for j in range(pr.k):
            q = o.spatial_candidate(W, H, centre, j, pr.radius, seed, 0, 0)
            if q >= 0:
                seen.add(int(cls[q]))
                merged += int(cls[q] in (0, 3))
        assert out[centre, 11] == 3.0 * merged
    assert seen == {0, 1, 2, 3}
