"""Pins of the oracle's reference path tracer (the converged images the
estimators are compared with) by closed forms:

* white furnace: a Lambertian plane under a uniform sky returns rho * L_sky
  for every sample (one bounce, then the sky);
* a convex sphere in a room whose walls emit L and reflect nothing returns
  rho_s * L exactly (one bounce to a wall, which ends the path);
* an enclosure of albedo a emitting L: every sample is L (1 + a + a^2 + a^3)
  plus an integer number of further L (each bounce the roulette keeps adds
  exactly L), and the mean matches L (1 - a^33) / (1 - a) (33 terms: the
  primary vertex and at most 32 bounces).
"""
import math

import numpy as np

import oracle as o
from paper_2108_05263_amd import scenegen as sg


def _cam(eye, look, W, H, fov=60.0):
    eye, look = np.asarray(eye, np.float64), np.asarray(look, np.float64)
    f = look - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return sg.Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32), right=r.astype(np.float32),
                     up=u.astype(np.float32), tan_half_fovy=float(np.float32(math.tan(math.radians(fov / 2)))),
                     width=W, height=H)


def test_furnace_plane_exact():
    sc = sg.furnace_plane()
    cam = sg.furnace_camera(24, 16)
    gb = o.gbuffer(sc, cam)
    pix = np.arange(24 * 16)
    out = o.path_trace(sc, gb, pix, 8, 3)
    hit = gb[:, 13] != o.MISS
    assert hit.any() and (~hit).any()
    want = np.asarray(sc.prims[0, 8:11], np.float64) * np.asarray(sc.sky, np.float64)
    assert np.allclose(out[hit], want, rtol=1e-12, atol=0)
    assert np.allclose(out[~hit], np.asarray(sc.sky, np.float64), rtol=0, atol=0)


def test_sphere_in_emitting_room_exact():
    sc = sg.emissive_room_sphere()
    cam = _cam((4.0, 4.0, 0.5), (4.0, 4.0, 4.0), 20, 20, 40.0)
    gb = o.gbuffer(sc, cam)
    out = o.path_trace(sc, gb, np.arange(400), 6, 5)
    on_sphere = gb[:, 13] == 0
    assert on_sphere.sum() > 50 and (~on_sphere).sum() > 20
    L = np.asarray(sc.wall_emit, np.float64)
    rho = np.asarray(sc.prims[0, 8:11], np.float64)
    assert np.allclose(out[on_sphere], rho * L, rtol=1e-12, atol=0)
    assert np.allclose(out[~on_sphere], L, rtol=1e-12, atol=0)


def test_albedo_enclosure_series():
    a = 0.6
    L = np.array([1.0, 2.0, 0.5])
    sc = sg.Scene(prims=np.zeros((0, 16), np.float32), has_room=True, room_lo=np.zeros(3, np.float32),
                  room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.full(3, a, np.float32),
                  sky=np.zeros(3, np.float32), eps=8e-4, wall_emit=L.astype(np.float32))
    a = float(np.float32(a))
    cam = _cam((4.0, 3.0, 2.0), (5.0, 4.0, 7.0), 24, 24)
    gb = o.gbuffer(sc, cam)
    spp = 32
    out = o.path_trace(sc, gb, np.arange(576), spp, 9)
    base = 1.0 + a + a * a + a ** 3
    K = (out / L - base) * spp                      # roulette survivors summed over the samples
    assert np.allclose(K, np.round(K), atol=1e-7)
    assert np.allclose(K[:, 0], K[:, 1]) and np.allclose(K[:, 0], K[:, 2])
    k = K[:, 0] / spp                                # per-pixel mean number of extra terms
    expect = (a ** 4 - a ** 33) / (1.0 - a)
    z = (k.mean() - expect) / (k.std(ddof=1) / math.sqrt(len(k)))
    assert abs(z) < 5.0, (k.mean(), expect, z)
    full = L * (1.0 - a ** 33) / (1.0 - a)
    assert np.allclose(out.mean(0), full, rtol=0.03)
