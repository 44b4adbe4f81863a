"""Pins of the oracle's glossy layer (Sec. 3.3: glossy L_DDGI+, Eq. 6, and
the specular recursion for shading, Eq. 7-8) by closed forms and by
quadrature of independent code paths:

* GGX at roughness 1 is the constant D = 1/pi, so at normal incidence the
  sampled directions are uniform on the sphere (density 1/(4 pi)) and half of
  them fall below the surface; at wo = wi = n, f_g = 1/(4 pi a^2);
* f_g is reciprocal;
* the sampling density integrates (hemisphere quadrature) to the fraction of
  samples the sampler returns above the surface;
* the sampler's estimate of the directional albedo (mean of f cos / pdf over a
  stratified grid of uniforms) matches the quadrature of f cos;
* with uniform probes (Q = q0 everywhere, unoccluded) the one-sample glossy
  part of L_DDGI+ averages to (q0 / 2) k_s A(wo): the 1/(2 pi) of Eq. 6 with
  E = pi Q;
* a glossy sphere (no diffuse albedo) in a room whose walls emit L and reflect
  nothing reflects k_s A(wo) L: the initial pass and shading estimate it
  without bias (mixture candidates, weights, full-BSDF target), and so does
  the reference path tracer;
* the shading recursion's two limits (it stops once the footprint exceeds
  a_0 c): threshold c = 0 always estimates the glossy sample from the probes
  (q0 / 2 per unit weight), c = infinity always traces it (and sees the
  emitting walls);
* a glossy code path with every k_s = 0 reproduces the Lambertian results.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as o
from paper_2108_05263_amd import scenegen as sg


def _hemi_grid(n, nt=360, nph=720):
    """Midpoint quadrature nodes over the hemisphere about n in (cos theta, phi):
    directions and solid-angle weights."""
    ct = (np.arange(nt) + 0.5) / nt
    ph = (np.arange(nph) + 0.5) / nph * 2 * np.pi
    C, P = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - C * C)
    n = np.asarray(n, float)
    t = np.cross(n, [1.0, 0, 0] if abs(n[0]) < 0.9 else [0, 1.0, 0])
    t /= np.linalg.norm(t)
    b = np.cross(n, t)
    d = (S * np.cos(P))[..., None] * t + (S * np.sin(P))[..., None] * b + C[..., None] * n
    w = np.full(C.shape, (1.0 / nt) * (2 * np.pi / nph))
    return d.reshape(-1, 3), w.reshape(-1), C.reshape(-1)


def _dir(theta_deg, phi_deg=30.0):
    t, p = math.radians(theta_deg), math.radians(phi_deg)
    return np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


N = np.array([0.0, 0.0, 1.0])


def test_ggx_closed_forms():
    # roughness 1: D = 1/pi, density 1/(4 pi) at normal incidence, f_g(n, n) = 1/(4 pi)
    for wi in (_dir(10), _dir(50), _dir(80)):
        f, pdf = o.ggx(N, N, wi, 1.0)
        assert pdf == pytest.approx(1.0 / (4 * np.pi), rel=1e-12)
    for a in (1.0, 0.5, 0.1):
        f, _ = o.ggx(N, N, N, a)
        assert f == pytest.approx(1.0 / (4 * np.pi * a * a), rel=1e-12)
    # half of the samples at normal incidence fall below the surface for a = 1
    u = (np.arange(200) + 0.5) / 200
    ok = sum(o.ggx_sample(N, N, 1.0, a, b) is not None for a in u for b in u[::10])
    assert ok / (200 * 20) == pytest.approx(0.5, abs=0.01)


def test_ggx_reciprocity():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = rng.uniform(0.02, 1.0)
        wo, wi = _dir(rng.uniform(0, 89), rng.uniform(0, 360)), _dir(rng.uniform(0, 89), rng.uniform(0, 360))
        assert o.ggx(N, wo, wi, a)[0] == pytest.approx(o.ggx(N, wi, wo, a)[0], rel=1e-12)


@pytest.mark.parametrize("a,theta", [(0.6, 0.0), (0.3, 40.0), (0.15, 70.0)])
def test_ggx_density_and_sampler_agree(a, theta):
    wo = _dir(theta)
    d, w, c = _hemi_grid(N)
    f, pdf = o.ggx_many(N, wo, d, a)
    mass = float((pdf * w).sum())                 # probability of a sample above the surface
    albedo = float((f * c * w).sum())             # A(wo) = int f_g cos
    u = (np.arange(300) + 0.5) / 300
    valid, est = 0, 0.0
    for u0 in u:
        for u1 in u[::3]:
            wi = o.ggx_sample(N, wo, a, u0, u1)
            if wi is None:
                continue
            valid += 1
            fv, pv = o.ggx(N, wo, wi, a)
            est += fv * wi[2] / pv
    n = 300 * 100
    assert valid / n == pytest.approx(mass, abs=5e-3)
    assert est / n == pytest.approx(albedo, rel=1e-2)
    assert 0.0 < albedo <= 1.0


def _uniform_probes(grid, q0):
    irr, dep = sg.empty_probe_textures(grid)
    irr[..., :3] = q0
    dep[..., 0] = 1e3
    dep[..., 1] = 1e6
    return irr, dep


def test_glossy_term_uniform_probes():
    """Eq. 6 with E = pi Q: the one-sample glossy part averages to (q0/2) k_s A(wo)."""
    cfg = sg.CONFIGS["tiny"]
    grid = sg.make_probe_grid(cfg)
    q0 = np.array([0.7, 1.3, 2.1])
    irr, dep = _uniform_probes(grid, q0)
    a, ks, wo = 0.35, 0.6, _dir(35.0)
    d, w, c = _hemi_grid(N)
    f, _ = o.ggx_many(N, wo, d, a)
    A = float((f * c * w).sum())
    pb = np.array([4.0, 4.0, 4.0])
    u = (np.arange(120) + 0.5) / 120
    acc = np.zeros(3)
    for u0 in u:
        for u1 in u:
            acc += o.glossy_term(grid, irr, dep, pb, N, wo, ks, a, u0, u1)
    acc /= len(u) ** 2
    assert np.allclose(acc, 0.5 * q0 * ks * A, rtol=1e-2)


def _glossy_sphere_room(ks, a, L):
    prims = sg.prim_records([sg.PRIM_SPHERE], [[4.0, 4.0, 4.0]], [[1.0, 0.0, 0.0]], [[0.0, 0.0, 0.0]],
                            [[0.0, 0.0, 0.0]], spec=[ks], rough=[a])
    return sg.Scene(prims=prims, has_room=True, room_lo=np.zeros(3, np.float32),
                    room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.zeros(3, np.float32),
                    sky=np.zeros(3, np.float32), eps=float(np.float32(8e-4)),
                    wall_emit=np.asarray(L, np.float32))


def _sphere_camera(W=16, H=16):
    eye, look = np.array([4.0, 4.6, 0.6]), np.array([4.0, 4.0, 4.0])
    f = (look - eye) / np.linalg.norm(look - eye)
    r = np.cross(f, [0.0, 1.0, 0.0])
    r /= np.linalg.norm(r)
    return sg.Camera(eye=eye.astype(np.float32), fwd=f.astype(np.float32), right=r.astype(np.float32),
                     up=np.cross(r, f).astype(np.float32),
                     tan_half_fovy=float(np.float32(math.tan(math.radians(12)))), width=W, height=H)


def _albedo_at(gb, p, eye, a):
    x, n = gb[p, 0:3], gb[p, 3:6]
    wo = np.asarray(eye, float) - x
    wo /= np.linalg.norm(wo)
    d, w, c = _hemi_grid(n, 240, 480)
    f, _ = o.ggx_many(n, wo, d, a)
    return float((f * c * w).sum())


def test_glossy_sphere_in_emitting_room_unbiased():
    """Initial pass + shading on a glossy sphere lit by emitting walls: the
    mean over seeds is k_s A(wo) L (no residual: walls are further than 1)."""
    ks, a, L = 0.8, 0.3, np.array([1.0, 2.0, 0.5])
    sc = _glossy_sphere_room(ks, a, L)
    cam = _sphere_camera()
    W, H = cam.width, cam.height
    gb = o.gbuffer(sc, cam)
    pix = np.nonzero(gb[:, 13] == 0)[0][::9][:8]
    assert len(pix) == 8
    grid = sg.make_probe_grid(sg.CONFIGS["tiny"])
    irr, dep = sg.empty_probe_textures(grid)
    pr = dataclasses.replace(sg.CONFIGS["tiny"].params, M=4)
    est = []
    for seed in range(1, 301):
        res, resid = o.resample_initial(sc, W, H, gb, grid, irr, dep, pr, seed, 0, pixels=pix, eye=cam.eye)
        img = o.shade(sc, W, H, gb, grid, irr, dep, res, resid, pr, pixels=pix, seed=seed, frame=0, eye=cam.eye)
        est.append(img[pix])
    est = np.asarray(est)
    for k, p in enumerate(pix):
        want = ks * _albedo_at(gb, p, cam.eye, a) * L
        m, se = est[:, k].mean(0), est[:, k].std(0, ddof=1) / math.sqrt(len(est))
        z = (m - want) / np.maximum(se, 1e-12)
        assert np.all(np.abs(z) < 5.0), (p, m, want, z)


def test_glossy_path_tracer_sphere_in_emitting_room():
    ks, a, L = 0.8, 0.3, np.array([1.0, 2.0, 0.5])
    sc = _glossy_sphere_room(ks, a, L)
    cam = _sphere_camera()
    gb = o.gbuffer(sc, cam)
    pix = np.nonzero(gb[:, 13] == 0)[0][::9][:6]
    out = o.path_trace(sc, gb, pix, 4000, 5, eye=cam.eye)
    for k, p in enumerate(pix):
        want = ks * _albedo_at(gb, p, cam.eye, a) * L
        assert np.allclose(out[k], want, rtol=0.03), (out[k], want)


def test_shading_recursion_limits():
    """c = 0 reads the probes for every glossy sample, c = inf traces it to the
    emitting walls: the glossy radiance of a selected sample on a glossy floor
    is k_s A q0/2 or k_s A L on average."""
    ks, a, L = 0.9, 0.2, np.array([1.5, 1.0, 0.5])
    prims = sg.prim_records([sg.PRIM_BOX, sg.PRIM_SPHERE], [[4.0, 0.5, 4.0], [4.0, 5.0, 4.0]],
                            [[3.5, 0.5, 3.5], [0.5, 0.0, 0.0]], [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]],
                            [[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], spec=[ks, 0.0], rough=[a, 1.0])
    sc = sg.Scene(prims=prims, has_room=True, room_lo=np.zeros(3, np.float32), room_hi=np.full(3, 8.0, np.float32),
                  wall_albedo=np.zeros(3, np.float32), sky=np.zeros(3, np.float32), eps=float(np.float32(8e-4)),
                  wall_emit=np.asarray(L, np.float32))
    # one pixel: the shading point on the sphere, its reservoir sample on the floor
    x, nx = np.array([4.0, 4.5, 4.0]), np.array([0.0, -1.0, 0.0])
    # the floor point's mirror direction heads away from the sphere, toward the walls
    y, ny = np.array([6.5, 1.0, 6.5]), np.array([0.0, 1.0, 0.0])
    W = H = 1
    gb = np.zeros((1, 14))
    gb[0, 0:3], gb[0, 3:6], gb[0, 6:9], gb[0, 12], gb[0, 13] = x, nx, [0.5, 0.5, 0.5], 3.0, 1
    grid = sg.make_probe_grid(sg.CONFIGS["tiny"])
    q0 = np.array([0.4, 0.8, 1.2])
    irr, dep = _uniform_probes(grid, q0)
    res = np.zeros((1, 14))
    res[0, 0:3], res[0, 3:6], res[0, 10], res[0, 11], res[0, 13] = y, ny, 1.0, 1.0, 0
    resid = np.zeros((1, 3))
    eye = np.array([2.0, 3.0, 2.0])                # below the sphere, facing x
    v = y - x
    d2 = v @ v
    w = v / math.sqrt(d2)
    geo = min((nx @ w) * (-(ny @ w)) / d2, 1.0)
    f_x = 0.5 / np.pi                                # the sphere is Lambertian
    wo_y = -w
    dd, ww, cc = _hemi_grid(ny, 240, 480)
    fg, _ = o.ggx_many(ny, wo_y, dd, a)
    A = float((fg * cc * ww).sum())
    for c, Lgl in ((0.0, q0 / 2), (float("inf"), L)):
        pr = dataclasses.replace(sg.CONFIGS["tiny"].params, foot_c=c, glossy_depth=8)
        acc = np.zeros(3)
        n = 4000
        for seed in range(n):
            acc += o.shade(sc, W, H, gb, grid, irr, dep, res, resid, pr, seed=seed, frame=0, eye=eye)[0]
        got = acc / n / (f_x * geo)
        # diffuse part of the floor is 0; its glossy part k_s A (L or q0/2)
        assert np.allclose(got, ks * A * Lgl, rtol=0.04), (c, got, ks * A * Lgl)


def test_glossy_path_reduces_to_lambertian():
    """Forcing the glossy code path on a scene without specular layers gives the
    Lambertian results (mixture = cosine sampling, f = rho/pi)."""
    cfg = sg.CONFIGS["tiny"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    cam = sg.make_camera(cfg, 0, 24, 24)
    gb = o.gbuffer(sc, cam)
    pr = cfg.params
    ref = o.resample_initial(sc, 24, 24, gb, grid, irr, dep, pr, 1, 0, eye=cam.eye)
    forced = o.ref._Scene(sc)
    forced.s.glossy = 1
    got = o.resample_initial(forced, 24, 24, gb, grid, irr, dep, pr, 1, 0, eye=cam.eye)
    assert np.array_equal(got[0][:, 12], ref[0][:, 12])          # same selections
    assert np.allclose(got[0], ref[0], rtol=1e-10, atol=1e-14)
    assert np.allclose(got[1], ref[1], rtol=1e-10, atol=1e-14)
    i1 = o.shade(sc, 24, 24, gb, grid, irr, dep, ref[0], ref[1], pr, eye=cam.eye)
    i2 = o.shade(forced, 24, 24, gb, grid, irr, dep, got[0], got[1], pr, eye=cam.eye)
    assert np.allclose(i1, i2, rtol=1e-10, atol=1e-14)


def _u(v):
    return (int(v) >> 8) * 2.0 ** -24


def _recursion_setup(extra_prims=False):
    """Shading point x on a Lambertian sphere (index 1), its reservoir sample y
    on a glossy floor (index 0, no diffuse albedo), an emitting room; with
    extra_prims a glossy slab (index 2) hangs below the ceiling."""
    ks, a, L = 0.9, 0.2, np.array([1.5, 1.0, 0.5])
    types = [sg.PRIM_BOX, sg.PRIM_SPHERE]
    cen, size = [[4.0, 0.5, 4.0], [4.0, 5.0, 4.0]], [[3.5, 0.5, 3.5], [0.5, 0.0, 0.0]]
    alb, spec, rough = [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]], [ks, 0.0], [a, 1.0]
    if extra_prims:
        types.append(sg.PRIM_BOX)
        cen.append([4.0, 7.25, 4.0])
        size.append([3.9, 0.25, 3.9])
        alb.append([0.0, 0.0, 0.0])
        spec.append(0.9)
        rough.append(0.3)
    prims = sg.prim_records(types, cen, size, alb, [[0.0, 0.0, 0.0]] * len(types), spec=spec, rough=rough)
    sc = sg.Scene(prims=prims, has_room=True, room_lo=np.zeros(3, np.float32), room_hi=np.full(3, 8.0, np.float32),
                  wall_albedo=np.zeros(3, np.float32), sky=np.zeros(3, np.float32), eps=float(np.float32(8e-4)),
                  wall_emit=np.asarray(L, np.float32))
    x, nx = np.array([4.0, 4.5, 4.0]), np.array([0.0, -1.0, 0.0])
    y, ny = (np.array([5.0, 1.0, 5.0]) if extra_prims else np.array([6.5, 1.0, 6.5])), np.array([0.0, 1.0, 0.0])
    gb = np.zeros((1, 14))
    gb[0, 0:3], gb[0, 3:6], gb[0, 6:9], gb[0, 12], gb[0, 13] = x, nx, [0.5, 0.5, 0.5], 3.0, 1
    res = np.zeros((1, 14))
    res[0, 0:3], res[0, 3:6], res[0, 10], res[0, 11], res[0, 13] = y, ny, 1.0, 1.0, 0
    eye = np.array([2.0, 3.0, 2.0])                # below the sphere, facing x
    grid = sg.make_probe_grid(sg.CONFIGS["tiny"])
    q0 = np.array([0.4, 0.8, 1.2])                 # probe colour: red/blue = 1/3; walls: 3
    irr, dep = _uniform_probes(grid, q0)
    return sc, gb, res, eye, grid, irr, dep, x, nx, y, ny


# red/blue ratios of the two outcomes, as stored (the tiny workload's FP32
# probe texels and scene records)
_PROBE_RB = float(np.float32(0.4)) / float(np.float32(1.2))
_WALL_RB = float(np.float32(1.5)) / float(np.float32(0.5))


def _a0(eye, x, nx):
    """Eq. 8: |x_0 - x_1|^2 / (4 pi cos) with x_0 the camera."""
    v = eye - x
    return (v @ v) / (4 * np.pi * (nx @ (v / np.linalg.norm(v))))


def _segment(a, b, nb, p):
    """One term of Eq. 7: sqrt(|a - b|^2 / (p <n_b, -w>)), w = direction a -> b."""
    v = b - a
    w = v / np.linalg.norm(v)
    return math.sqrt((v @ v) / (p * (-(nb @ w))))


def _shade1(sc, gb, grid, irr, dep, res, c, seed, eye):
    pr = dataclasses.replace(sg.CONFIGS["tiny"].params, foot_c=c, glossy_depth=8)
    return o.shade(sc, 1, 1, gb, grid, irr, dep, res, np.zeros((1, 3)), pr, seed=seed, frame=0, eye=eye)[0]


def test_shading_recursion_threshold_first_segment():
    """Eq. 7-8 at the selected sample: the footprint of x -> y, with p_1 the
    cosine density of the Lambertian x, against a_0 of the camera-x segment.
    The threshold c* = a(x y) / a_0 is computed here by hand; just below it
    every glossy sample at y is read from the probes (probe colour), just
    above it every one is traced to the emitting walls (wall colour)."""
    sc, gb, res, eye, grid, irr, dep, x, nx, y, ny = _recursion_setup()
    w = (y - x) / np.linalg.norm(y - x)
    p1 = (nx @ w) / np.pi
    c_star = _segment(x, y, ny, p1) ** 2 / _a0(eye, x, nx)
    assert 10.0 < c_star < 1000.0                  # far from 1: a missing square root shows
    seen = {0.99: 0, 1.01: 0}
    for f, ratio in ((0.99, _PROBE_RB), (1.01, _WALL_RB)):
        for seed in range(40):
            out = _shade1(sc, gb, grid, irr, dep, res, f * c_star, seed, eye)
            if out[2] == 0.0:
                continue                           # the lobe sample fell below the floor
            seen[f] += 1
            assert out[0] / out[2] == pytest.approx(ratio, rel=1e-9), (f, seed, out)
    assert min(seen.values()) >= 20


def test_shading_recursion_threshold_sums_segments():
    """The footprint of a two-segment path x -> y -> z is the square of the
    SUM of the segments' square roots (Eq. 7), the second segment's density
    being the glossy lobe's at y.  z lies on a glossy slab; for each seed the
    threshold c* = a(x y z) / a_0 is computed from that seed's own lobe sample
    at y: just below it z reads the probes, just above it z's own lobe sample
    is traced (to a wall, for the seeds used)."""
    sc, gb, res, eye, grid, irr, dep, x, nx, y, ny = _recursion_setup(extra_prims=True)
    w = (y - x) / np.linalg.norm(y - x)
    s1 = _segment(x, y, ny, (nx @ w) / np.pi)
    a0 = _a0(eye, x, nx)
    wo_y = -w
    a_y, a_z = 0.2, 0.3
    used = 0
    for seed in range(200):
        u = o.philox(seed, [0, 0, 16, 1])                     # y is recursion depth 1
        wi = o.ggx_sample(ny, wo_y, a_y, _u(u[0]), _u(u[1]))
        if wi is None:
            continue
        hit, t, prim, nz = o.closest_hit(sc, y + float(np.float32(8e-4)) * ny, wi)
        if not hit or prim != 2:
            continue
        z = y + float(np.float32(8e-4)) * ny + t * wi
        s2 = _segment(y, z, nz, o.ggx(ny, wo_y, wi, a_y)[1])
        # z's own lobe sample (depth 2) must reach a wall for the traced case to show the wall colour
        u2 = o.philox(seed, [0, 0, 16, 2])
        wo_z = (y - z) / np.linalg.norm(y - z)
        wz = o.ggx_sample(nz, wo_z, a_z, _u(u2[0]), _u(u2[1]))
        if wz is None:
            continue
        hit2, _, prim2, _ = o.closest_hit(sc, z + float(np.float32(8e-4)) * nz, wz)
        if not hit2 or prim2 < 3:
            continue
        c_star = (s1 + s2) ** 2 / a0
        assert c_star > 1.05 * s1 * s1 / a0                     # y itself traces at both c
        below = _shade1(sc, gb, grid, irr, dep, res, 0.99 * c_star, seed, eye)
        above = _shade1(sc, gb, grid, irr, dep, res, 1.01 * c_star, seed, eye)
        assert below[0] / below[2] == pytest.approx(_PROBE_RB, rel=1e-9), (seed, below)
        assert above[0] / above[2] == pytest.approx(_WALL_RB, rel=1e-9), (seed, above)
        # the sum of squares (no cross term) would put the threshold elsewhere
        assert abs((s1 * s1 + s2 * s2) / a0 / c_star - 1.0) > 0.02
        used += 1
    assert used >= 10, used
