"""Pins of the oracle's ray casting, samplers and primary vertices.

* analytic hits (sphere through its centre, axis-aligned box faces, room walls);
* closest hit == first root found by an independent signed-distance ray march
  (numpy, a different formulation of the same geometry);
* cosine sampler: cos(theta) = sqrt(1 - u1) exactly, orthonormal basis,
  E[cos] = 2/3, chi^2 of the cos^2 distribution;
* uniform-sphere sampler moments;
* pinhole camera: pixel centres map to the documented directions.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as o
from paper_2108_05263_amd import scenegen as g


def _scene(prims, room=False, lo=(0, 0, 0), hi=(8, 8, 8)):
    return g.Scene(prims=prims, has_room=room, room_lo=np.asarray(lo, np.float32),
                   room_hi=np.asarray(hi, np.float32), wall_albedo=np.full(3, 0.8, np.float32),
                   sky=np.ones(3, np.float32), eps=1e-3)


def test_sphere_through_centre():
    sc = _scene(g.prim_records([0], [[1.0, 2.0, 3.0]], [[0.5, 0, 0]], [[.5] * 3], [[0] * 3]))
    o_ = np.array([1.0, 2.0, -4.0])
    d = np.array([0.0, 0.0, 1.0])
    hit, t, prim, n = o.closest_hit(sc, o_, d)
    assert hit and prim == 0
    assert t == pytest.approx(7.0 - 0.5, abs=1e-12)
    assert np.allclose(n, [0, 0, -1])
    # from the centre outward: t = r, normal faces the ray (inward)
    hit, t, prim, n = o.closest_hit(sc, [1.0, 2.0, 3.0], [0.0, 1.0, 0.0])
    assert hit and t == pytest.approx(0.5) and np.allclose(n, [0, -1, 0])


def test_box_faces_and_inside():
    sc = _scene(g.prim_records([1], [[0.0, 0.0, 0.0]], [[1.0, 2.0, 3.0]], [[.5] * 3], [[0] * 3]))
    for axis, half in enumerate([1.0, 2.0, 3.0]):
        for sgn in (-1, 1):
            org = np.zeros(3)
            org[axis] = sgn * 10.0
            d = np.zeros(3)
            d[axis] = -sgn
            d += 1e-9 * np.array([1, 2, 3])  # avoid exactly zero components
            d /= np.linalg.norm(d)
            hit, t, prim, n = o.closest_hit(sc, org, d)
            assert hit and t == pytest.approx(10.0 - half, abs=1e-6)
            ne = np.zeros(3)
            ne[axis] = sgn
            assert np.allclose(n, ne)
    hit, t, prim, n = o.closest_hit(sc, [0.0, 0.0, 0.0], [0.6, 0.8, 0.0])
    assert hit and t == pytest.approx(min(1.0 / 0.6, 2.0 / 0.8))
    assert np.allclose(n, [-1, 0, 0])


def test_room_walls_and_indices():
    sc = _scene(g.prim_records([0], [[4.0, 4.0, 4.0]], [[1.0, 0, 0]], [[.5] * 3], [[0] * 3]),
                room=True)
    hit, t, prim, n = o.closest_hit(sc, [1.0, 1.0, 1.0], [0.0, -1.0, 0.0])
    assert hit and t == pytest.approx(1.0) and prim == 1 + 2 * 1 + 0 and np.allclose(n, [0, 1, 0])
    hit, t, prim, n = o.closest_hit(sc, [1.0, 1.0, 1.0], [0.0, 0.0, 1.0])
    assert hit and t == pytest.approx(7.0) and prim == 1 + 2 * 2 + 1 and np.allclose(n, [0, 0, -1])


def test_tie_goes_to_lower_index():
    sc = _scene(g.prim_records([0, 0], [[0, 0, 5.0]] * 2, [[1.0, 0, 0]] * 2, [[.5] * 3] * 2,
                               [[0] * 3] * 2))
    hit, t, prim, n = o.closest_hit(sc, [0, 0, 0], [0, 0, 1.0])
    assert hit and prim == 0


def _sdf(scene, p):
    """Signed distance to the union of the scene's primitives and the room
    walls (inside the room the wall distance is the distance to the boundary)."""
    rec = scene.prims
    types = rec.view(np.uint32)[:, 3]
    best = np.full(p.shape[0], np.inf)
    for i in range(len(rec)):
        c, s = rec[i, 0:3].astype(np.float64), rec[i, 4:7].astype(np.float64)
        if types[i] == 0:
            dist = np.linalg.norm(p - c, axis=1) - s[0]
        else:
            q = np.abs(p - c) - s
            dist = np.linalg.norm(np.maximum(q, 0.0), axis=1) + np.minimum(q.max(axis=1), 0.0)
        best = np.minimum(best, np.abs(dist))
    if scene.has_room:
        lo, hi = scene.room_lo.astype(np.float64), scene.room_hi.astype(np.float64)
        wall = np.minimum((p - lo).min(axis=1), (hi - p).min(axis=1))
        best = np.minimum(best, np.abs(wall))
    return best


def _march(scene, org, d, tmax=200.0):
    """Unsigned sphere tracing: first t where the distance falls below 1e-9."""
    t = np.zeros(org.shape[0])
    done = np.zeros(org.shape[0], bool)
    for _ in range(4000):
        p = org + t[:, None] * d
        dist = _sdf(scene, p)
        hit = dist < 1e-9
        done |= hit
        t = np.where(done, t, t + dist)
        if np.all(done | (t > tmax)):
            break
    return np.where(done, t, np.inf)


def test_closest_hit_matches_sdf_march():
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    rng = np.random.default_rng(3)
    n = 300
    org = rng.uniform(0.3, 7.7, (n, 3))
    # keep origins outside every primitive (the march is unsigned)
    ok = _sdf(sc, org) > 0.05
    rec, types = sc.prims, sc.prims.view(np.uint32)[:, 3]
    for i in range(len(rec)):
        c, s = rec[i, 0:3].astype(np.float64), rec[i, 4:7].astype(np.float64)
        if types[i] == 0:
            ok &= np.linalg.norm(org - c, axis=1) > s[0]
    org = org[ok]
    d = rng.normal(size=(len(org), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tm = _march(sc, org, d)
    for i in range(len(org)):
        hit, t, prim, nrm = o.closest_hit(sc, org[i], d[i])
        assert hit
        assert t == pytest.approx(tm[i], abs=1e-6), i
        assert np.dot(nrm, d[i]) <= 0.0


def test_visibility_agrees_with_closest_hit():
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg)
    gb = o.gbuffer(sc, cam)
    rng = np.random.default_rng(5)
    hits = np.where(gb[:, 13] != o.MISS)[0]
    for _ in range(200):
        a, b = rng.choice(hits, 2, replace=False)
        pa, na, pb, nb = gb[a, 0:3], gb[a, 3:6], gb[b, 0:3], gb[b, 3:6]
        v_ab = o.visible(sc, pa, na, pb, nb)
        v_ba = o.visible(sc, pb, nb, pa, na)
        assert v_ab == v_ba
        org = pa + sc.eps * na
        tgt = pb + sc.eps * nb
        dist = np.linalg.norm(tgt - org)
        hit, t, _, _ = o.closest_hit(sc, org, (tgt - org) / dist)
        assert v_ab == (not (hit and t < dist))


def test_cosine_sampler():
    rng = np.random.default_rng(11)
    normals = rng.normal(size=(8, 3))
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    normals = np.vstack([normals, [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0]]])
    for n in normals:
        us = rng.random((2000, 2))
        w = np.array([o.cosine_dir(n, u0, u1) for u0, u1 in us])
        assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
        cos = w @ n
        assert np.allclose(cos, np.sqrt(1.0 - us[:, 1]), atol=1e-12)
        # azimuth: the tangent-plane part rotates by 2*pi*u0 (orthonormal basis)
        tan = w - cos[:, None] * n
        a0 = o.cosine_dir(n, 0.0, 0.5) - math.sqrt(0.5) * n
        for (u0, u1), t in zip(us[:50], tan[:50]):
            ang = math.acos(np.clip(np.dot(t, a0) / (np.linalg.norm(t) * np.linalg.norm(a0)), -1, 1))
            expect = 2 * math.pi * u0
            expect = min(expect, 2 * math.pi - expect)
            assert ang == pytest.approx(expect, abs=1e-6)
    # distribution: cos^2 theta is uniform, E[cos] = 2/3
    us = rng.random((20000, 2))
    n = normals[0]
    cos = np.array([o.cosine_dir(n, u0, u1) @ n for u0, u1 in us])
    assert abs(cos.mean() - 2.0 / 3.0) < 0.01
    hist, _ = np.histogram(cos ** 2, bins=20, range=(0, 1))
    assert stats.chisquare(hist).pvalue > 1e-4


def test_sphere_sampler():
    rng = np.random.default_rng(12)
    us = rng.random((20000, 2))
    w = np.array([o.sphere_dir(u0, u1) for u0, u1 in us])
    assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
    assert np.allclose(w[:, 2], 1.0 - 2.0 * us[:, 0])
    assert np.all(np.abs(w.mean(0)) < 0.03)
    assert np.allclose((w ** 2).mean(0), 1.0 / 3.0, atol=0.02)


def test_gbuffer_camera_rays():
    cfg = g.CONFIGS["tiny"]
    sc = g.make_scene(cfg)
    cam = g.make_camera(cfg)
    gb = o.gbuffer(sc, cam)
    W, H = cam.width, cam.height
    eye = cam.eye.astype(np.float64)
    for p in [0, W - 1, (H - 1) * W, W * H - 1, (H // 2) * W + W // 2 + 3]:
        i, j = p % W, p // W
        sx = (2 * (i + 0.5) / W - 1) * cam.tan_half_fovy * (W / H)
        sy = (1 - 2 * (j + 0.5) / H) * cam.tan_half_fovy
        d = cam.fwd.astype(np.float64) + sx * cam.right.astype(np.float64) + sy * cam.up.astype(np.float64)
        d /= np.linalg.norm(d)
        v = gb[p, 0:3] - eye
        t = np.linalg.norm(v)
        assert np.allclose(v / t, d, atol=1e-12)
        assert gb[p, 12] == pytest.approx(t * np.dot(d, cam.fwd.astype(np.float64)))
        hit, th, prim, _ = o.closest_hit(sc, eye, d)
        assert hit and th == pytest.approx(t) and prim == int(gb[p, 13])
    # the camera sits inside the room: every primary ray hits something
    assert np.all(gb[:, 13] != o.MISS)
