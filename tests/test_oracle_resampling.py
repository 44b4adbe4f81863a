"""Pins of the oracle's resampling passes and shading.

* white furnace: a Lambertian plane of albedo rho under a uniform sky L gives
  rho * L in every pixel exactly, through initial RIS, temporal reuse and
  spatial reuse (all samples are sky directions with constant RIS weight);
* a convex sphere inside a room whose walls emit L and reflect nothing gives
  rho * L on the sphere exactly after initial RIS + shading (area-measure
  samples, geometry term, pdf conversion, contribution weight, shadow ray);
* the residual transport vanishes when no geometry term exceeds G_max;
* with a static camera the reprojection maps every pixel onto itself;
* spatial neighbours are uniform in the disk of the given radius;
* unbiasedness: per-pixel mean over seeds of the full estimator (initial,
  spatial and temporal reuse, bounded term + residual) agrees with a
  brute-force uniform-hemisphere Monte Carlo integral (z-test, Bonferroni);
* MAPE (Sec. 4) on hand-computed values.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as o
from paper_2108_05263_amd import scenegen as g
from paper_2108_05263_amd import scenegen as sg


def _params(**kw):
    p = g.Params(M=8, k=3, n_spatial=1, radius=4.0, temporal=False)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_white_furnace_plane_full_pipeline():
    rho = np.array([0.5, 0.7, 0.9], np.float32)
    L = np.array([1.0, 2.0, 3.0], np.float32)
    sc = g.furnace_plane(albedo=rho, sky=L)
    cam = g.furnace_camera(24, 16)
    grid = g.probe_grid((2, 2, 2), (-1, -1, -1), 1.0)
    irr, dep = g.empty_probe_textures(grid)
    pr = _params(M=8, k=4, n_spatial=2, temporal=True)
    seq = o.Sequence(sc, grid, irr, dep, pr, seed=7)
    for f in range(3):
        img, st = seq.frame(cam, f)
        gb = st["gbuffer"]
        on = gb[:, 13] != o.MISS
        assert on.sum() > 100 and (~on).sum() > 10
        expect = (rho.astype(np.float64) * L.astype(np.float64))
        assert np.allclose(img[on], expect, rtol=1e-12)
        assert np.allclose(img[~on], L.astype(np.float64), rtol=0)
        if f > 0:
            assert "temporal" in st
            # every reservoir counts all merged candidates and visibility never fails
            assert np.all(st["spatial1"][on, 11] > pr.M)


def test_furnace_sphere_in_emissive_room():
    rho = np.array([0.3, 0.6, 0.9], np.float32)
    L = np.array([2.0, 1.0, 0.5], np.float32)
    sc = g.emissive_room_sphere(albedo=rho, radiance=L)
    cfg = g.CONFIGS["tiny"]
    cam = g.make_camera(cfg, width=32, height=32)
    cam.eye = np.array([4.0, 4.0, 0.5], np.float32)
    cam.fwd = np.array([0.0, 0.0, 1.0], np.float32)
    cam.right = np.array([-1.0, 0.0, 0.0], np.float32)
    cam.up = np.array([0.0, 1.0, 0.0], np.float32)
    grid = g.probe_grid((2, 2, 2), (0, 0, 0), 4.0)
    irr, dep = g.empty_probe_textures(grid)
    pr = _params(M=16, n_spatial=0)
    seq = o.Sequence(sc, grid, irr, dep, pr, seed=3)
    img, st = seq.frame(cam, 0)
    gb = st["gbuffer"]
    sphere = gb[:, 13] == 0
    assert sphere.sum() > 50
    assert np.allclose(img[sphere], rho.astype(np.float64) * L.astype(np.float64), rtol=1e-11)
    assert np.allclose(img[~sphere], L.astype(np.float64), rtol=0)
    assert np.all(st["resid"] == 0.0)


def _tiny_setup(W=16, H=16):
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg, width=W, height=H)
    grid = g.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    return cfg, sc, cam, grid, irr, dep


def test_residual_vanishes_without_bounding():
    cfg, sc, cam, grid, irr, dep = _tiny_setup(32, 32)
    gb = o.gbuffer(sc, cam)
    _, resid = o.resample_initial(sc, 32, 32, gb, grid, irr, dep, _params(g_max=1e30), 5, 0)
    assert np.all(resid == 0.0)
    _, resid = o.resample_initial(sc, 32, 32, gb, grid, irr, dep, _params(g_max=1.0), 5, 0)
    assert np.any(resid > 0.0)


def test_static_reprojection_is_identity():
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg, width=40, height=30)
    gb = o.gbuffer(sc, cam)
    for p in range(0, 40 * 30, 7):
        assert o.reproject(cam, gb[p, 0:3]) == p


def test_spatial_candidates_uniform_in_disk():
    W = H = 201
    p = 100 * W + 100
    R = 30.0
    dx, dy = [], []
    for j in range(20000):
        q = o.spatial_candidate(W, H, p, j % 5, R, 1000 + j // 5, 0, 0)
        if q < 0:
            continue
        dx.append(q % W - 100)
        dy.append(q // W - 100)
    dx, dy = np.array(dx, np.float64), np.array(dy, np.float64)
    r2 = dx * dx + dy * dy
    assert r2.max() <= (R + 1) ** 2
    n = len(dx)
    # uniform disk of radius R, rounded to the lattice: zero mean,
    # E[r^2] = R^2/2 + 2/12 (rounding adds 1/12 per axis), isotropic angle
    assert abs(dx.mean()) < 4 * R / 2 / math.sqrt(n) and abs(dy.mean()) < 4 * R / 2 / math.sqrt(n)
    assert r2.mean() == pytest.approx(R * R / 2 + 1.0 / 6.0, rel=0.02)
    # bins centred on the axes, so lattice points on an axis sit mid-bin
    ang = np.mod(np.arctan2(dy, dx) + math.pi / 8, 2 * math.pi)
    hist, _ = np.histogram(ang, bins=8, range=(0.0, 2 * math.pi))
    assert stats.chisquare(hist).pvalue > 1e-4


def test_determinism():
    cfg, sc, cam, grid, irr, dep = _tiny_setup(16, 16)
    a, _ = o.Sequence(sc, grid, irr, dep, cfg.params, 3).frame(cam, 0)
    b, _ = o.Sequence(sc, grid, irr, dep, cfg.params, 3).frame(cam, 0)
    assert np.array_equal(a, b)


def _over_seeds(sc, cam, grid, irr, dep, pr, seeds, frames=1):
    lw = np.array([0.2126, 0.7152, 0.0722])
    imgs = []
    for s in seeds:
        seq = o.Sequence(sc, grid, irr, dep, pr, s)
        for f in range(frames):
            img, st = seq.frame(cam, f)
        imgs.append(img @ lw)
    return np.array(imgs), st["gbuffer"]


@pytest.mark.parametrize("variant", ["initial", "spatial", "temporal", "shadow"])
def test_unbiased_against_brute_force(variant):
    """Mean of the whole estimator over seeds vs brute-force Monte Carlo."""
    W = H = 12
    nseeds = 160
    if variant == "shadow":
        # sharp occlusion between neighbours: the normalisation must test visibility
        W = H = 16
        nseeds = 800
        sc, cam = g.shadow_scene(), g.shadow_camera(W, H)
        grid = g.probe_grid((2, 2, 2), (-1, -1, -1), 1.0)
        irr, dep = g.empty_probe_textures(grid)
    else:
        cfg, sc, cam, grid, irr, dep = _tiny_setup(W, H)
    if variant == "shadow":
        pr, frames = _params(M=4, k=4, n_spatial=2, radius=6.0), 1
    elif variant == "initial":
        pr, frames = _params(M=8, n_spatial=0), 1
    elif variant == "spatial":
        pr, frames = _params(M=4, k=3, n_spatial=2, radius=3.0), 1
    else:
        pr, frames = _params(M=4, k=3, n_spatial=1, radius=3.0, temporal=True), 2
    lum, gb = _over_seeds(sc, cam, grid, irr, dep, pr, range(100, 100 + nseeds), frames)
    mean, se = lum.mean(0), lum.std(0, ddof=1) / math.sqrt(nseeds)
    pix = np.arange(W * H)
    lw = np.array([0.2126, 0.7152, 0.0722])
    ref = o.brute_force(sc, W, H, gb, grid, irr, dep, pix, 6000, seed=99) @ lw
    # brute-force standard error from a second independent run
    ref2 = o.brute_force(sc, W, H, gb, grid, irr, dep, pix, 6000, seed=98) @ lw
    se_ref = np.abs(ref2 - ref) / math.sqrt(2)
    active = (gb[:, 13] != o.MISS) & (gb[:, 6:9].max(1) > 0)
    z = (mean - ref)[active] / np.sqrt(se[active] ** 2 + se_ref[active] ** 2 + 1e-12)
    # per pixel: Bonferroni at family-wise 1e-3 over the active pixels
    zc = stats.norm.isf(1e-3 / (2 * active.sum()))
    assert np.mean(np.abs(z) > zc) <= 0.01, (np.sort(np.abs(z))[-5:], zc)
    # whole image: the sum over active pixels, with its own standard errors
    tot = lum[:, active].sum(1)
    se_tot = tot.std(ddof=1) / math.sqrt(nseeds)
    se_ref_tot = abs((ref2 - ref)[active].sum()) / math.sqrt(2) + 1e-3 * ref[active].sum()
    z_tot = (tot.mean() - ref[active].sum()) / math.hypot(se_tot, se_ref_tot)
    assert abs(z_tot) < 4.0, (z_tot, tot.mean() / ref[active].sum() - 1)


def test_mape_hand_values():
    v = np.array([1.0, 0.0, 2.0, 0.5])
    r = np.array([1.0, 0.01, 1.0, 0.99])
    expect = (0.0 + 0.01 / 0.02 + 1.0 / 1.01 + 0.49 / 1.0) / 4
    assert o.mape(v, r) == pytest.approx(expect, rel=1e-14)


def _sphere_over_plane():
    """A Lambertian plane (top face y = 0) under a black sky, lit only by an
    emissive sphere wholly above it; a camera looking down at the plane."""
    rho = np.array([0.6, 0.5, 0.4], np.float32)
    Le = np.array([[30.0, 20.0, 10.0], [200.0, 300.0, 400.0]], np.float32)
    r = np.array([0.8, 1.5])
    c = np.array([[0.3, 2.4, 0.8], [25.0, 3.0, 0.8]])
    # the far sphere stays above the horizon and out of the near one's shadow
    # for every plane point the camera sees
    prims = sg.prim_records([sg.PRIM_BOX, sg.PRIM_SPHERE, sg.PRIM_SPHERE], [[0.0, -1.0, 0.0], c[0], c[1]],
                            [[50.0, 1.0, 50.0], [r[0], 0, 0], [r[1], 0, 0]], [rho, [0, 0, 0], [0, 0, 0]],
                            [[0, 0, 0], Le[0], Le[1]])
    sc = sg.Scene(prims=prims, has_room=False, room_lo=np.zeros(3, np.float32), room_hi=np.zeros(3, np.float32),
                  wall_albedo=np.zeros(3, np.float32), sky=np.zeros(3, np.float32), eps=float(np.float32(1e-3)))
    eye, look = np.array([0.3, 3.0, -2.5]), np.array([0.3, 0.0, 1.0])
    f = (look - eye) / np.linalg.norm(look - eye)
    rt = np.cross(f, [0.0, 1.0, 0.0])
    rt /= np.linalg.norm(rt)
    cam = sg.Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32), right=rt.astype(np.float32),
                    up=np.cross(rt, f).astype(np.float32),
                    tan_half_fovy=float(np.float32(math.tan(math.radians(25.0)))), width=12, height=10)
    return sc, cam, rho.astype(np.float64), Le.astype(np.float64), r, c


def test_emitter_candidates_unbiased_closed_form():
    """Emitter-sampled candidates with balance-heuristic weights: a sphere of
    radiance L_e and radius r wholly above a plane gives irradiance
    pi L_e (r/d)^2 cos(theta) (a classic closed form), so each plane pixel
    converges to rho sum_e L_e (r_e/d_e)^2 cos(theta_e) for two unoccluded
    emissive spheres.  Per-pixel z-test over seeds; the emitter candidates
    must also cut the variance."""
    sc, cam, rho, Le, r, c = _sphere_over_plane()
    W, H = cam.width, cam.height
    gb = o.gbuffer(sc, cam)
    grid = sg.probe_grid((2, 2, 2), (-8.0, -1.0, -8.0), 8.0)
    irr, dep = sg.empty_probe_textures(grid)
    plane = (gb[:, 13] == 0) & (np.abs(gb[:, 4] - 1.0) < 1e-12)
    assert plane.sum() > 60
    x = gb[plane, 0:3]
    exact = np.zeros((len(x), 3))
    for e in range(2):
        v = c[e] - x
        d = np.linalg.norm(v, axis=1)
        exact += rho[None, :] * Le[e][None, :] * ((r[e] / d) ** 2 * (v[:, 1] / d))[:, None]
    S = 300
    var = {}
    for M, ml in ((4, 0), (4, 4), (2, 8)):
        pr = sg.Params(M=M, M_light=ml, k=0, n_spatial=0, temporal=False)
        vals = np.zeros((S, int(plane.sum()), 3))
        for s in range(S):
            res, resid = o.resample_initial(sc, W, H, gb, grid, irr, dep, pr, 1000 + s, 0)
            vals[s] = o.shade(sc, W, H, gb, grid, irr, dep, res, resid, pr)[plane]
        mean, sd = vals.mean(0), vals.std(0, ddof=1)
        var[ml] = float((sd ** 2).mean())
        if ml == 0:
            continue    # cosine candidates alone almost never reach the far sphere: no z-test
        z = (mean - exact) / (sd / math.sqrt(S) + 1e-12)
        # Bonferroni over the plane pixels and channels at family-wise 1e-3
        assert np.abs(z).max() < 5.0, (M, ml, np.abs(z).max())
    assert var[4] < 0.5 * var[0], var


def test_subsampling_draws_on_the_pattern():
    """Subsampling (Sec. 6): pixel (x, y) draws candidates in frame f iff
    (x + y + f) % n == 0.  Drawing pixels get exactly the reservoirs of the
    plain pass (same counters); the others an empty reservoir (M = 0, W = 0);
    every pixel keeps its residual (candidate 0)."""
    W, H = 12, 10
    cfg, sc, cam, grid, irr, dep = _tiny_setup(W, H)
    gb = o.gbuffer(sc, cam)
    active = (gb[:, 13] != o.MISS) & (gb[:, 6:9].max(1) > 0)
    for n, frame in ((2, 0), (3, 5), (1, 2)):
        full, rfull = o.resample_initial(sc, W, H, gb, grid, irr, dep, _params(M=6), 4, frame)
        sub, rsub = o.resample_initial(sc, W, H, gb, grid, irr, dep, _params(M=6, subsample=n), 4, frame)
        x, y = np.arange(W * H) % W, np.arange(W * H) // W
        draws = (x + y + frame) % n == 0
        assert np.array_equal(sub[draws], full[draws])
        assert np.all(sub[active & ~draws, 11] == 0) and np.all(sub[~draws, 10] == 0)
        assert np.array_equal(rsub, rfull)
        assert (active & ~draws).any() or n == 1
