"""Pins of the oracle's probe volume: octahedral map, gutters, query, update.

* octahedral encode/decode round trip; texel centres; bilinear fetch at a
  texel centre returns the texel;
* gutters make the fetch continuous across the octahedral folds (a smooth
  function sampled at texel centres is reproduced everywhere, edges included);
* with the backface and visibility terms switched off and a constant value
  per probe, the query equals scipy's trilinear RegularGridInterpolator;
* constant textures give a constant query whatever the weights;
* visibility limits (probe fully visible / fully hidden);
* update: empty space under sky L gives E/pi = L and depth = (d_max, d_max^2)
  exactly; the Lambertian plane of albedo 1 under sky L is a fixed point with
  E = pi L on the plane; hysteresis follows a^k; a texel converges to the
  analytic irradiance of a probe above a black plane.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle as o
from paper_2108_05263_amd import scenegen as g


def _dirs(n, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_octahedral_round_trip():
    for v in _dirs(500):
        uv = o.oct_encode(v)
        assert 0.0 <= uv[0] <= 1.0 and 0.0 <= uv[1] <= 1.0
        assert np.allclose(o.oct_decode(uv), v, atol=1e-12)
    for v in ([0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, -1.0, 0]):
        assert np.allclose(o.oct_decode(o.oct_encode(v)), v, atol=1e-12)


def _smooth(v):
    return np.array([1.0 + 0.5 * v[0], 2.0 + 0.3 * v[1] - 0.2 * v[2], 0.5 + 0.4 * v[2] ** 2])


def _tile_from(fn, N):
    P = N + 2
    tile = np.zeros((P * P, 3))
    for ty in range(N):
        for tx in range(N):
            d = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
            tile[(ty + 1) * P + tx + 1] = fn(d)
    return o.fill_gutter(tile, N)


@pytest.mark.parametrize("N", [8, 16])
def test_fetch_at_texel_centres(N):
    tile = _tile_from(_smooth, N)
    for ty in range(N):
        for tx in range(N):
            d = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
            assert np.allclose(o.tile_fetch(tile, N, d), tile[(ty + 1) * (N + 2) + tx + 1], atol=1e-12)


def test_gutters_make_fetch_continuous():
    N = 16
    tile = _tile_from(_smooth, N)
    # directions next to the equator and the -z pole (where the folds are),
    # and both sides of every fold, must reproduce the smooth function
    worst = 0.0
    for v in _dirs(3000, 4):
        if abs(v[2]) > 0.15 and v[2] > -0.85:
            continue
        worst = max(worst, np.abs(o.tile_fetch(tile, N, v) - _smooth(v)).max())
    assert worst < 0.05
    # a pure fold test: mirrored directions across the z=0 edge agree
    for v in _dirs(500, 5):
        v = np.array([v[0], v[1], 1e-9])
        v /= np.linalg.norm(v)
        w = np.array([v[0], v[1], -1e-9])
        w /= np.linalg.norm(w)
        assert np.allclose(o.tile_fetch(tile, N, v), o.tile_fetch(tile, N, w), atol=1e-6)


def _f16(x):
    """binary16 rounding (numpy's float16 conversion), the precision of the
    stored texels of a binary16 probe volume, back in float64"""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def _store(x, texel):
    """a texel value as a probe volume of the given format stores it (the
    FP32 volume: as given, the oracle keeping full precision)"""
    return _f16(x) if texel == "f16" else np.asarray(x, np.float64)


TEXELS = pytest.mark.parametrize("texel", ["f32", "f16"])


def _grid(dims=(4, 3, 5), spacing=1.5, texel="f32"):
    return g.probe_grid(dims, (0.0, 0.0, 0.0), spacing, texel=texel)


@TEXELS
def test_query_equals_trilinear_when_weights_off(texel):
    grid = _grid(texel=texel)
    P = grid.count
    rng = np.random.default_rng(8)
    vals = rng.uniform(0.1, 3.0, (P, 3))
    irr = np.repeat(vals[:, None, :], (grid.irr_res + 2) ** 2, axis=1)
    dep = rng.uniform(0.0, 2.0, (P, (grid.dep_res + 2) ** 2, 2))
    nx, ny, nz = grid.dims
    s = float(grid.spacing[0])
    axes = [(np.arange(n) + 0.5) * s for n in (nx, ny, nz)]
    # irradiance texels are read at their storage precision
    grid_vals = _store(vals, texel).reshape(nz, ny, nx, 3).transpose(2, 1, 0, 3)
    interp = RegularGridInterpolator(axes, grid_vals)
    pts = np.stack([rng.uniform(a[0], a[-1], 400) for a in axes], axis=1)
    nrm = _dirs(400, 9)
    q = o.probe_query(grid, irr, dep, pts, nrm, flags=3)
    assert np.allclose(q, interp(pts), atol=1e-12, rtol=1e-12)
    # outside the probe box the grid coordinate clamps to the border probes
    out = np.array([[-5.0, 1.0, 2.0]])
    q_out = o.probe_query(grid, irr, dep, out, nrm[:1], flags=3)
    clamp = np.array([[axes[0][0], 1.0, 2.0]])
    assert np.allclose(q_out, interp(clamp), atol=1e-12)


@TEXELS
def test_query_constant_textures_give_constant(texel):
    grid = _grid(texel=texel)
    P = grid.count
    rng = np.random.default_rng(10)
    irr = np.zeros((P, (grid.irr_res + 2) ** 2, 3)) + np.array([0.7, 1.1, 2.3])
    dep = rng.uniform(0.0, 2.5, (P, (grid.dep_res + 2) ** 2, 1))
    dep = np.concatenate([dep, dep ** 2 + rng.uniform(0, 0.5, dep.shape)], axis=2)
    pts = rng.uniform(0.0, 7.0, (300, 3))
    q = o.probe_query(grid, irr, dep, pts, _dirs(300, 3))
    assert np.allclose(q, _store([0.7, 1.1, 2.3], texel), atol=1e-12)
    if texel == "f16":
        assert not np.allclose(q, [0.7, 1.1, 2.3], atol=1e-6)   # the texels' precision shows


def test_query_visibility_limits():
    grid = _grid((2, 2, 2), 2.0)
    P = grid.count
    vals = np.arange(P, dtype=np.float64)[:, None] * np.ones(3) + 1.0
    irr = np.repeat(vals[:, None, :], (grid.irr_res + 2) ** 2, axis=1)
    nd = (grid.dep_res + 2) ** 2
    far = np.zeros((P, nd, 2))
    far[..., 0], far[..., 1] = 100.0, 100.0 ** 2
    pts = np.random.default_rng(2).uniform(1.0, 3.0, (100, 3))
    nrm = _dirs(100, 6)
    # every probe sees farther than the query point: visibility 1
    assert np.allclose(o.probe_query(grid, irr, far, pts, nrm, 0),
                       o.probe_query(grid, irr, far, pts, nrm, 2), atol=1e-12)
    # probe 0 is hidden (mean distance 0, variance at the floor): with the
    # backface term off its weight collapses to ~1e-6 x trilinear and the query
    # becomes the trilinear blend of the seven others, renormalised
    hidden = far.copy()
    hidden[0] = 0.0
    q = o.probe_query(grid, irr, hidden, pts, nrm, flags=1)
    f = (pts - 1.0) / 2.0
    num = np.zeros(len(pts))
    den = np.zeros(len(pts))
    for c in range(1, 8):
        ox, oy, oz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        t = ((f[:, 0] if ox else 1 - f[:, 0]) * (f[:, 1] if oy else 1 - f[:, 1])
             * (f[:, 2] if oz else 1 - f[:, 2]))
        num += t * vals[c, 0]
        den += t
    assert np.allclose(q[:, 0], num / den, rtol=1e-5)


# --------------------------------------------------------------------------
# probe update
# --------------------------------------------------------------------------
def _open_scene(prims=None, sky=(1.5, 0.5, 2.0)):
    if prims is None:
        prims = np.zeros((0, 16), np.float32)
    return g.Scene(prims=prims, has_room=False, room_lo=np.zeros(3, np.float32),
                   room_hi=np.zeros(3, np.float32), wall_albedo=np.zeros(3, np.float32),
                   sky=np.asarray(sky, np.float32), eps=1e-3)


@TEXELS
def test_update_empty_space_under_sky(texel):
    sky = np.array([1.5, 0.5, 2.0], np.float32)
    sc = _open_scene(sky=sky)
    grid = _grid((2, 2, 2), 1.0, texel)
    irr, dep = g.empty_probe_textures(grid)
    i2, d2 = o.probe_update(sc, grid, irr, dep, rays=128, hysteresis=0.0, sharpness=50.0, seed=3,
                            frame=0)
    assert np.allclose(i2, sky.astype(np.float64), rtol=1e-14, atol=0)
    # depth texels: mean d_max and variance 0 (binary16: mean square rebuilt
    # from the stored mean)
    assert np.allclose(d2[..., 0], _store(grid.d_max, texel), rtol=1e-14)
    assert np.allclose(d2[..., 1], _store(grid.d_max, texel) ** 2, rtol=1e-13)


@TEXELS
def test_update_plane_fixed_point_gives_pi_L(texel):
    L = np.array([0.8, 1.3, 2.1], np.float32)
    plane = g.prim_records([1], [[0.0, -1.0, 0.0]], [[1000.0, 1.0, 1000.0]], [[1.0, 1.0, 1.0]],
                           [[0, 0, 0]])
    sc = _open_scene(plane, sky=L)
    grid = g.probe_grid((3, 3, 3), (-1.5, 0.0, -1.5), 1.0, texel=texel)
    irr, dep = g.empty_probe_textures(grid)
    irr[..., :3] = L
    dep[..., 0], dep[..., 1] = 1.0, 1.0
    i2, d2 = o.probe_update(sc, grid, irr, dep, rays=64, hysteresis=0.0, sharpness=50.0, seed=1,
                            frame=0)
    # the stored texels are L at the storage precision: the sky rays bring
    # L, the plane rays the stored value, and every mean of the two rounds
    # back to it
    Lh = _store(L, texel)
    assert np.allclose(i2, Lh, rtol=1e-12)
    # query on the plane: Q = E/pi = L (as stored), i.e. E = pi L
    pts = np.array([[0.1, 0.0, 0.2], [-0.7, 0.0, 0.4]])
    q = o.probe_query(grid, i2, d2, pts, [[0, 1.0, 0]] * 2)
    assert np.allclose(math.pi * q, math.pi * Lh, rtol=1e-12)


@TEXELS
def test_update_hysteresis_geometric(texel):
    sky = np.array([2.0, 2.0, 2.0], np.float32)
    sc = _open_scene(sky=sky)
    grid = _grid((2, 2, 2), 1.0, texel)
    irr, dep = g.empty_probe_textures(grid)
    irr = irr[..., :3].astype(np.float64) + 0.5
    dep = dep.astype(np.float64)
    a = 0.9
    expect = 0.5
    for k in range(1, 6):
        irr, dep = o.probe_update(sc, grid, irr, dep, 64, a, 50.0, 1, k)
        # a^k 0.5 + (1 - a^k) 2, each step's blend stored at the storage precision
        expect = float(_store(a * expect + (1 - a) * 2.0, texel))
        assert np.allclose(irr, expect, rtol=1e-12)
    assert abs(expect - (a ** 5 * 0.5 + (1 - a ** 5) * 2.0)) < 2e-3


def test_update_texel_converges_to_analytic_irradiance():
    # probe above an infinite black plane under sky L: a texel with direction n
    # at angle theta from +y sees E/pi = L (1 + cos theta) / 2
    L = 1.0
    plane = g.prim_records([1], [[0.0, -1.0, 0.0]], [[1000.0, 1.0, 1000.0]], [[0, 0, 0]],
                           [[0, 0, 0]])
    sc = _open_scene(plane, sky=(L, L, L))
    grid = g.probe_grid((1, 1, 1), (-0.5, 0.0, -0.5), 1.0)
    irr, dep = g.empty_probe_textures(grid)
    i2, _ = o.probe_update(sc, grid, irr, dep, 4096, 0.0, 50.0, 5, 0)
    N = grid.irr_res
    errs = []
    for ty in range(N):
        for tx in range(N):
            n = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
            got = i2[0, (ty + 1) * (N + 2) + tx + 1, 0]
            errs.append(got - L * (1 + n[1]) / 2)
    assert np.max(np.abs(errs)) < 0.03
    assert abs(np.mean(errs)) < 0.006


def _random_tile(N, C, seed):
    P = N + 2
    rng = np.random.default_rng(seed)
    tile = np.zeros((P * P, C))
    for ty in range(N):
        for tx in range(N):
            tile[(ty + 1) * P + tx + 1] = rng.uniform(0, 1, C)
    return o.fill_gutter(tile, N)


@pytest.mark.parametrize("N", [8, 16])
def test_fetch_continuous_across_border_folds(N):
    """The outer border of the octahedral square is a fold: directions just on
    either side of the planes x=0 and y=0 (lower hemisphere) map to mirrored
    points of the same border.  With correct gutters the bilinear fetch agrees
    on both sides for ANY texel values; near -z all four corners meet."""
    tile = _random_tile(N, 3, N)
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, z = rng.uniform(-1, 1), -rng.uniform(0.05, 1.0)
        for axis in (0, 1):
            vp = np.zeros(3)
            vp[1 - axis], vp[2] = a, z
            vm = vp.copy()
            vp[axis], vm[axis] = 1e-10, -1e-10
            vp /= np.linalg.norm(vp)
            vm /= np.linalg.norm(vm)
            assert np.allclose(o.tile_fetch(tile, N, vp), o.tile_fetch(tile, N, vm), atol=1e-7)
    corner = [o.tile_fetch(tile, N, np.array([sx * 1e-9, sy * 1e-9, -1.0]))
              for sx in (-1, 1) for sy in (-1, 1)]
    for c in corner[1:]:
        assert np.allclose(c, corner[0], atol=1e-7)


def test_update_depth_clamped_and_probe_centred():
    # one probe at the centre of a 6^3 room: texels that face a wall read
    # a depth mean close to 3 (the cos^50 lobe is narrow); all depths <= d_max
    sc = g.Scene(prims=np.zeros((0, 16), np.float32), has_room=True,
                 room_lo=np.zeros(3, np.float32), room_hi=np.full(3, 6.0, np.float32),
                 wall_albedo=np.zeros(3, np.float32), sky=np.zeros(3, np.float32), eps=1e-3)
    grid = g.probe_grid((1, 1, 1), (0, 0, 0), 6.0)
    grid.d_max = 100.0
    irr, dep = g.empty_probe_textures(grid)
    _, d2 = o.probe_update(sc, grid, irr, dep, 4096, 0.0, 50.0, 2, 0)
    N = grid.dep_res
    for ty in range(N):
        for tx in range(N):
            n = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
            if np.max(np.abs(n)) > 0.97:
                m = d2[0, (ty + 1) * (N + 2) + tx + 1, 0]
                assert 3.0 <= m < 3.3, (n, m)
    grid.d_max = 2.0
    _, d3 = o.probe_update(sc, grid, irr, dep, 256, 0.0, 50.0, 2, 0)
    assert np.all(d3[..., 0] <= 2.0 + 1e-12) and np.all(d3[..., 1] <= 4.0 + 1e-12)


def test_update_emission_enters_undiffused():
    # a probe enclosed by an emissive sphere of radiance Le (albedo 0): every
    # probe ray returns Le itself, so every texel stores E/pi = Le (Eq. 5)
    le = np.array([3.0, 5.0, 7.0], np.float32)
    prims = g.prim_records([0], [[0.5, 0.5, 0.5]], [[2.0, 0, 0]], [[0, 0, 0]], [le])
    sc = g.Scene(prims=prims, has_room=False, room_lo=np.zeros(3, np.float32),
                 room_hi=np.zeros(3, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.zeros(3, np.float32), eps=1e-3)
    grid = g.probe_grid((1, 1, 1), (0, 0, 0), 1.0)
    irr, dep = g.empty_probe_textures(grid)
    i2, d2 = o.probe_update(sc, grid, irr, dep, 128, 0.0, 50.0, 2, 0)
    assert np.allclose(i2, le.astype(np.float64), rtol=1e-13)


def test_query_backface_prefers_probes_in_front():
    # query at the centre of a cubic cell, normal pointing at probe c: the
    # eight weights are ((1 + cos)/2)^2 + 0.2 with cos in {1, 1/3, -1/3, -1}
    grid = _grid((2, 2, 2), 2.0)
    P = grid.count
    nd = (grid.dep_res + 2) ** 2
    far = np.zeros((P, nd, 2))
    far[..., 0], far[..., 1] = 100.0, 100.0 ** 2
    p = np.array([[2.0, 2.0, 2.0]])
    for c in range(8):
        vals = np.zeros(P)
        vals[c] = 1.0
        irr = np.repeat((vals[:, None] * np.ones(3))[:, None, :], (grid.irr_res + 2) ** 2, axis=1)
        corner = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1]) * 2.0 + 1.0
        n = (corner - p[0]) / np.linalg.norm(corner - p[0])
        q = o.probe_query(grid, irr, far, p, n[None], 0)[0, 0]
        w = [((1 + cs) / 2) ** 2 + 0.2 for cs in (1, 1 / 3, 1 / 3, 1 / 3, -1 / 3, -1 / 3, -1 / 3, -1)]
        assert q == pytest.approx(w[0] / sum(w), rel=1e-12)
        q_back = o.probe_query(grid, irr, far, p, -n[None], 0)[0, 0]
        assert q_back == pytest.approx(w[-1] / sum(w), rel=1e-12)


@TEXELS
def test_query_chebyshev_weight(texel):
    # two probes along x; probe 0 stores depth moments (mu, mu^2 + s2) in every
    # texel, probe 1 sees far.  The query's value recovers probe 0's
    # visibility weight, which must be the cubed one-sided Chebyshev bound
    # s2 / (s2 + (r - mu)^2) when r > mu, and 1 when r <= mu.
    grid = g.probe_grid((2, 1, 1), (0, 0, 0), 2.0, texel=texel)
    nd = (grid.dep_res + 2) ** 2
    irr = np.zeros((2, (grid.irr_res + 2) ** 2, 3))
    irr[1] = 1.0
    # the last case's variance (1e-3) is below the binary16 step of its mean
    # square (1.44: 2^-10), so a rounded mean square would lose it
    for mu, s2, xq in [(0.3, 0.04, 1.6), (0.5, 0.01, 2.2), (0.2, 0.2, 1.4), (1.0, 0.05, 1.5), (1.2, 1e-3, 2.25)]:
        dep = np.zeros((2, nd, 2))
        dep[0, :, 0], dep[0, :, 1] = mu, mu * mu + s2
        dep[1, :, 0], dep[1, :, 1] = 100.0, 1e4
        p = np.array([[xq, 1.0, 1.0]])
        q = o.probe_query(grid, irr, dep, p, [[0, 1.0, 0]], flags=1)[0, 0]
        t1 = (xq - 1.0) / 2.0
        t0 = 1.0 - t1
        v0 = t1 * (1.0 - q) / (t0 * q)
        r = xq - 1.0
        # the texels hold the mean and the variance at the storage precision
        mu, s2 = float(_store(mu, texel)), float(_store((mu * mu + s2) - mu * mu, texel))
        cheb = 1.0 if r <= mu else (s2 / (s2 + (r - mu) ** 2)) ** 3
        assert v0 == pytest.approx(max(cheb, 1e-6), rel=1e-9), (mu, s2, xq)


@TEXELS
def test_distance_heuristic_single_ray(texel):
    """Emission heuristic of the probe update (Sec. 3.2): a probe at the
    centre of a cube room whose walls emit L and reflect nothing, one update
    ray of length t: every irradiance texel facing the ray holds L (t / (t +
    s d_b))^2, with d_b the probe's backward mean depth clipped to its cell.
    Here the cell is the room, so a backward depth beyond the walls clips to
    t and the factor is 1/(1+s)^2 whatever the direction; slider 0 leaves L."""
    L = np.array([0.7, 1.1, 1.9], np.float32)
    sc = g.Scene(prims=np.zeros((0, 16), np.float32), has_room=True, room_lo=np.zeros(3, np.float32),
                 room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.zeros(3, np.float32), eps=8e-4, wall_emit=L)
    grid = g.probe_grid((1, 1, 1), (0.0, 0.0, 0.0), 8.0, texel=texel)
    N = grid.irr_res
    Ld = L.astype(np.float64)
    for frame in range(6):
        u = o.philox(3, [0, frame, 9, 0])
        w = o.sphere_dir(float(u[0] >> 8) * 2.0 ** -24, float(u[1] >> 8) * 2.0 ** -24)
        t = float(np.min(4.0 / np.abs(w)))
        for mu_b, s, factor in ((100.0, 0.7, 1.0 / 1.7 ** 2), (1.5, 0.7, (t / (t + 0.7 * 1.5)) ** 2),
                                (1.5, 0.0, 1.0)):
            irr, dep = g.empty_probe_textures(grid)
            dep[..., 0], dep[..., 1] = mu_b, mu_b * mu_b
            i2, _ = o.probe_update(sc, grid, irr, dep, 1, 0.0, 50.0, 3, frame, slider=s)
            T = i2.reshape(N + 2, N + 2, 3)[1:N + 1, 1:N + 1]
            facing, checked = 0, 0
            for ty in range(N):
                for tx in range(N):
                    nt = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
                    if np.dot(nt, w) > 1e-9:
                        assert np.allclose(T[ty, tx], _store(Ld * factor, texel), rtol=1e-12), (frame, mu_b, s)
                        facing += 1
                    elif np.dot(nt, w) < -1e-9:
                        assert np.all(T[ty, tx] == 0.0)
                    checked += 1
            assert facing > 10


@TEXELS
def test_distance_heuristic_reads_the_backward_direction(texel):
    """Same room; the probe's depth tile says 'far' (beyond the cell) for
    directions with z > 0 and 1.5 for z < 0, so the factor tells which
    direction was read: the backward one, -w."""
    L = np.array([1.0, 2.0, 3.0], np.float32)
    sc = g.Scene(prims=np.zeros((0, 16), np.float32), has_room=True, room_lo=np.zeros(3, np.float32),
                 room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.zeros(3, np.float32),
                 sky=np.zeros(3, np.float32), eps=8e-4, wall_emit=L)
    grid = g.probe_grid((1, 1, 1), (0.0, 0.0, 0.0), 8.0, texel=texel)
    N, Nd = grid.irr_res, grid.dep_res
    irr, dep = g.empty_probe_textures(grid)
    tile = np.zeros((Nd + 2, Nd + 2, 2))
    for ty in range(Nd):
        for tx in range(Nd):
            d = o.oct_decode([(tx + 0.5) / Nd, (ty + 0.5) / Nd])
            mu = 100.0 if d[2] > 0 else 1.5
            tile[ty + 1, tx + 1] = (mu, mu * mu)
    dep[0] = o.fill_gutter(tile.reshape(-1, 2), Nd).reshape(-1, 2)
    s, seen = 0.5, {True: 0, False: 0}
    for frame in range(40):
        u = o.philox(7, [0, frame, 9, 0])
        w = o.sphere_dir(float(u[0] >> 8) * 2.0 ** -24, float(u[1] >> 8) * 2.0 ** -24)
        if abs(w[2]) < 0.4:
            continue
        t = float(np.min(4.0 / np.abs(w)))
        far = -w[2] > 0
        factor = 1.0 / (1.0 + s) ** 2 if far else (t / (t + s * 1.5)) ** 2
        i2, _ = o.probe_update(sc, grid, irr, dep, 1, 0.0, 50.0, 7, frame, slider=s)
        T = i2.reshape(N + 2, N + 2, 3)[1:N + 1, 1:N + 1]
        best = max(((ty, tx) for ty in range(N) for tx in range(N)),
                   key=lambda c: np.dot(o.oct_decode([(c[1] + 0.5) / N, (c[0] + 0.5) / N]), w))
        assert np.allclose(T[best], _store(L.astype(np.float64) * factor, texel), rtol=1e-12), (frame, far)
        seen[far] += 1
    assert seen[True] >= 3 and seen[False] >= 3


def _lobe_means(nt, s, fn, nu=1000, nph=1000):
    """Means of fn(direction) and fn(direction)^2 under the normalised lobe
    max(0, nt.w)^s dw, by midpoint quadrature in (u, phi) with cos(theta) =
    u^(1/(s+1)): the substitution makes the lobe's weight uniform in u."""
    u = (np.arange(nu) + 0.5) / nu
    ph = (np.arange(nph) + 0.5) / nph * 2 * np.pi
    U, P = np.meshgrid(u, ph, indexing="ij")
    c = U ** (1.0 / (s + 1.0))
    sn = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    nt = np.asarray(nt, float)
    t = np.cross(nt, [1.0, 0, 0] if abs(nt[0]) < 0.9 else [0, 1.0, 0])
    t /= np.linalg.norm(t)
    b = np.cross(nt, t)
    w = (sn * np.cos(P))[..., None] * t + (sn * np.sin(P))[..., None] * b + c[..., None] * nt
    f = fn(w.reshape(-1, 3))
    return float(f.mean()), float((f * f).mean())


@TEXELS
@pytest.mark.parametrize("sharp", [2.0, 50.0])
def test_update_depth_moments_above_plane(sharp, texel):
    """Both depth moments of Sec. 3.2's mean visibility (the Chebyshev test
    reads their difference as a variance).  Probes at height h above an
    infinite plane: a ray of direction w meets the plane at h / (-w_y), so the
    stored moments must be the lobe means of d and d^2 with d = min(h / (-w_y),
    d_max) below the horizon and d_max above it, computed here by quadrature.
    At sharpness 2 the variance is large, so storing the squared mean in place
    of the mean square fails."""
    plane = g.prim_records([1], [[0.0, -1.0, 0.0]], [[1000.0, 1.0, 1000.0]], [[0.0, 0.0, 0.0]],
                           [[0, 0, 0]])
    sc = _open_scene(plane, sky=(0.0, 0.0, 0.0))
    grid = g.probe_grid((8, 1, 8), (-4.0, 0.5, -4.0), 1.0, texel=texel)
    h, D = 1.0, float(grid.d_max)
    irr, dep = g.empty_probe_textures(grid)
    _, d2 = o.probe_update(sc, grid, irr, dep, 4096, 0.0, sharp, 11, 0)
    N = grid.dep_res

    def depth(w):
        down = w[:, 1] < 0
        d = np.full(len(w), D)
        d[down] = np.minimum(h / -w[down, 1], D)
        return d

    worst = 0.0
    for ty in range(0, N, 3):
        for tx in range(0, N, 3):
            nt = o.oct_decode([(tx + 0.5) / N, (ty + 0.5) / N])
            want1, want2 = _lobe_means(nt, sharp, depth)
            got = d2[:, (ty + 1) * (N + 2) + tx + 1, :]          # 64 independent probes
            for k, want in ((0, want1), (1, want2)):
                m = got[:, k].mean()
                se = got[:, k].std(ddof=1) / math.sqrt(len(got))
                if se < 1e-12:                                   # all sky: d_max^k, stored as
                    assert m == pytest.approx(_store(D, texel) ** (k + 1), rel=1e-9), (nt, k, m, want)
                    continue
                # quadrature error at this resolution is below 1e-5 relative; a
                # binary16 volume stores the mean and variance to a relative step of 2^-11
                z = (m - want) / se
                worst = max(worst, abs(z))
                assert abs(m - want) < 5.0 * se + (1e-5 + 2.0 ** -10) * want, (nt, k, m, want, se)
    assert worst > 0.0
    if sharp == 2.0:
        # the downward texels see a real spread of depths: E[d^2] - E[d]^2 > 0
        nt = np.array([0.0, -1.0, 0.0])
        m1, m2 = _lobe_means(nt, sharp, depth)
        var = m2 - m1 * m1
        assert var > 0.05


# --------------------------------------------------------------------------
# binary16 irradiance texels
# --------------------------------------------------------------------------
def test_round_half_matches_numpy_float16():
    """o_round_half against numpy's float64 -> float16 conversion: normal and
    subnormal ranges, ties (to even), the largest finite value and overflow."""
    rng = np.random.default_rng(31)
    xs = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000),
                         [0.0, -0.0, 65504.0, 65519.99, 65520.0, -65520.0, 1e6, 2.0 ** -24, 2.0 ** -25,
                          3 * 2.0 ** -26, 2.0 ** -14, 2.0 ** -14 * (1 - 2.0 ** -11), 1 + 2.0 ** -11,
                          1 + 3 * 2.0 ** -11, 2049.0, 2051.0]])
    with np.errstate(over="ignore"):
        want = xs.astype(np.float16).astype(np.float64)
    got = np.array([o.round_half(x) for x in xs])
    assert np.array_equal(got, want)


def test_update_stores_binary16_and_query_reads_binary16():
    """In a binary16 volume the update stores irradiance texels that are
    binary16 values; the query reads a caller's arbitrary tile at that
    precision (a tile of 1 + 2^-12, which rounds to 1, queries as exactly 1)."""
    sky = np.array([0.3, 0.7, 1.9], np.float32)
    sc = _open_scene(sky=sky)
    grid = _grid((2, 2, 2), 1.0, "f16")
    irr, dep = g.empty_probe_textures(grid)
    i2, d2 = o.probe_update(sc, grid, irr, dep, rays=32, hysteresis=0.25, sharpness=50.0, seed=5, frame=0)
    # empty space under the sky: every texel is 0.75 L, stored at binary16
    want = 0.75 * sky.astype(np.float64)
    assert np.array_equal(i2, _f16(i2))
    assert np.allclose(i2, want, rtol=1e-3) and not np.allclose(i2, want, rtol=1e-6)
    tile = np.full_like(i2, 1.0 + 2.0 ** -12)
    q = o.probe_query(grid, tile, d2, [[0.7, 0.6, 0.8]], [[0.0, 1.0, 0.0]])
    assert np.array_equal(q, [[1.0, 1.0, 1.0]])


def test_fp32_volume_keeps_full_precision():
    """In an FP32 volume the oracle keeps texels at full precision: the
    same update stores 0.75 L (to the rounding of its ray sums), and the
    tile of 1 + 2^-12 queries as itself."""
    sky = np.array([0.3, 0.7, 1.9], np.float32)
    sc = _open_scene(sky=sky)
    grid = _grid((2, 2, 2), 1.0, "f32")
    irr, dep = g.empty_probe_textures(grid)
    i2, d2 = o.probe_update(sc, grid, irr, dep, rays=32, hysteresis=0.25, sharpness=50.0, seed=5, frame=0)
    want = 0.75 * sky.astype(np.float64)
    assert np.allclose(i2, want, rtol=1e-14, atol=0)
    assert not np.allclose(i2, _f16(want), rtol=1e-6)
    tile = np.full_like(i2, 1.0 + 2.0 ** -12)
    q = o.probe_query(grid, tile, d2, [[0.7, 0.6, 0.8]], [[0.0, 1.0, 0.0]])
    assert np.allclose(q, 1.0 + 2.0 ** -12, rtol=1e-15, atol=0)


def test_binary16_blend_below_half_a_step_is_lost():
    """The cost of binary16 texels under hysteresis: a stored irradiance of 1
    blended at h = 0.97 toward 1.01 moves by 3e-4, less than half the binary16
    step at 1 (2^-11), so a binary16 volume keeps 1 while an FP32 volume
    stores 0.97 + 0.03 x 1.01."""
    sky = np.array([1.01, 1.01, 1.01], np.float32)
    sc = _open_scene(sky=sky)
    for texel in ("f32", "f16"):
        grid = _grid((2, 2, 2), 1.0, texel)
        irr, dep = g.empty_probe_textures(grid)
        irr = irr[..., :3].astype(np.float64) + 1.0
        i2, _ = o.probe_update(sc, grid, irr, dep.astype(np.float64), 64, 0.97, 50.0, 1, 0)
        want = 0.97 + 0.03 * float(sky[0])
        if texel == "f16":
            assert np.all(i2 == 1.0)
        else:
            assert np.allclose(i2, want, rtol=1e-12) and np.all(i2 > 1.0)
