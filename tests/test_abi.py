"""The C-ABI library loads, exports every symbol include/gi.h declares, and
rejects bad arguments on the host before launching anything (no GPU needed:
validation never touches the device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2108_05263_amd import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gi():
    if libbuild.is_stale():
        libbuild.build()
    from paper_2108_05263_amd import gi as m
    m.load()
    return m


def test_exports_every_declared_symbol(gi):
    hdr = open(os.path.join(ROOT, "include", "gi.h")).read()
    declared = set(re.findall(r"^\w[\w\s\*]*?\b(gi_\w+)\s*\(", hdr, re.M))
    assert declared >= {"gi_trace_gbuffer", "gi_probe_update", "gi_resample_initial",
                        "gi_resample_temporal", "gi_resample_spatial", "gi_shade"}
    lib = gi.load()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(gi.EXPORTS)


def test_library_built_from_these_sources(gi):
    """The library carries the hash of the sources and flags it was built
    from; loading refuses a library built from others."""
    from paper_2108_05263_amd import build
    assert gi.load().gi_build_hash().decode() == build.source_hash() == build.built_hash()


def test_binding_fails_loudly_without_the_library(gi, monkeypatch):
    """No fallback: with the library missing, or built from other sources,
    loading raises instead of running anything else."""
    from paper_2108_05263_amd import build
    monkeypatch.setattr(gi, "_lib", None)
    monkeypatch.setattr(gi, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libgi.so"))
    with pytest.raises(gi.GiError, match="not built"):
        gi.load()
    monkeypatch.undo()
    monkeypatch.setattr(gi, "_lib", None)
    monkeypatch.setattr(build, "source_hash", lambda *a, **k: "0" * 16)
    with pytest.raises(gi.GiError, match="other sources"):
        gi.load()
    monkeypatch.undo()
    assert gi.load() is not None


def test_status_strings(gi):
    lib = gi.load()
    for s in range(7):
        assert lib.gi_status_string(s)
    assert lib.gi_status_string(99) == b"unknown status"


def _null():
    return C.c_void_p(0)


def test_validation_rejects_before_launch(gi):
    lib = gi.load()
    s = gi.GiScene()
    cam = gi.GiCamera()
    cam.width, cam.height = 4, 4
    g = gi.GiGBuffer()
    g.width, g.height = 4, 4
    # null pointers
    assert lib.gi_trace_gbuffer(None, C.byref(cam), C.byref(g), None) == 1
    assert lib.gi_trace_gbuffer(C.byref(s), C.byref(cam), C.byref(g), None) == 1
    # shape mismatch
    g.pos_depth = g.nrm_prim = g.albedo = g.emit = 16
    g.width = 5
    assert lib.gi_trace_gbuffer(C.byref(s), C.byref(cam), C.byref(g), None) == 2
    # parameters out of range
    r = gi.GiReservoirs()
    r.width, r.height = 4, 4
    r.y_W, r.n_wsum, r.L_M, r.tag_prim = 16, 32, 48, 64
    g.width = 4
    pr = gi.GiProbes()
    pr.dims = (C.c_uint32 * 3)(2, 2, 2)
    pr.irr_res, pr.dep_res = 8, 16
    pr.spacing = gi.F3(1.0, 1.0, 1.0)
    pr.irr, pr.dep = 80, 96
    pp = gi.GiParams()
    pp.M, pp.k, pp.radius, pp.g_max, pp.m_cap = 33, 1, 1.0, 1.0, 20.0
    pp.subsample = 1
    resid = C.c_void_p(112)
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 3
    pp.M = 8
    # emitter candidates beyond the 32-candidate limit, subsample 0
    pp.M_light = 25
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 3
    pp.M_light, pp.subsample = 24, 0
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 3
    pp.subsample = 1
    # emitter list: too long, or naming a primitive that does not exist
    s.n_emitters = 33
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 2
    s.n_emitters, s.emitters[0] = 1, 5
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 3
    s.n_emitters = 0
    pr.irr_res = 4
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 2
    pr.irr_res = 8
    # an unknown texel format
    pr.texel = 2
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 3
    assert lib.gi_probe_query(C.byref(pr), 0, resid, resid, resid, None) == 3
    pr.texel = 0
    # aliasing output and input reservoirs
    assert lib.gi_resample_spatial(C.byref(s), C.byref(g), C.byref(r), C.byref(pp), 0, C.byref(r),
                                   1, 0, None) == 4
    # probe update: rays out of range, aliasing
    pu = gi.GiProbeParams(0, 0.5, 50.0, 0.0)
    pr2 = gi.GiProbes()
    C.pointer(pr2)[0] = pr
    pr2.irr, pr2.dep = 128, 144
    assert lib.gi_probe_update(C.byref(s), C.byref(pr), C.byref(pr2), C.byref(pu), 1, 0, None) == 3
    pu.rays, pu.distance_slider = 64, -1.0
    assert lib.gi_probe_update(C.byref(s), C.byref(pr), C.byref(pr2), C.byref(pu), 1, 0, None) == 3
    pu.distance_slider = 0.0
    pu.rays = 64
    assert lib.gi_probe_update(C.byref(s), C.byref(pr), C.byref(pr), C.byref(pu), 1, 0, None) == 4
    # input and output volumes of different texel formats
    pr2.texel = 1
    assert lib.gi_probe_update(C.byref(s), C.byref(pr), C.byref(pr2), C.byref(pu), 1, 0, None) == 3
    pr2.texel = 0


def test_accel_builder_lists_overlapping_cells(gi):
    from paper_2108_05263_amd import scenegen as sg
    cfg = sg.CONFIGS["hd"]
    sc = sg.make_scene(cfg)
    lib = gi.load()
    lo, hi = sc.bounds()
    res = (C.c_uint32 * 3)(*cfg.grid_res)
    ncell = int(np.prod(cfg.grid_res))
    start = np.zeros(ncell + 1, np.uint32)
    n = C.c_uint32()
    rec = np.ascontiguousarray(sc.prims)
    st = lib.gi_accel_build_host(rec.ctypes.data_as(C.c_void_p), len(rec), gi._f3(lo), gi._f3(hi), res,
                                 start.ctypes.data_as(C.c_void_p), None, 0, C.byref(n))
    assert st == 2 and n.value > len(rec)
    items = np.zeros(n.value, np.uint32)
    st = lib.gi_accel_build_host(rec.ctypes.data_as(C.c_void_p), len(rec), gi._f3(lo), gi._f3(hi), res,
                                 start.ctypes.data_as(C.c_void_p), items.ctypes.data_as(C.c_void_p),
                                 len(items), C.byref(n))
    assert st == 0 and start[-1] == n.value
    # every primitive appears in the cell that contains its centre, ids increase per cell
    cs = (hi - lo) / np.array(cfg.grid_res)
    for i in range(len(rec)):
        c = np.clip(((rec[i, 0:3] - lo) / cs).astype(int), 0, np.array(cfg.grid_res) - 1)
        cell = c[0] + cfg.grid_res[0] * (c[1] + cfg.grid_res[1] * c[2])
        assert i in items[start[cell]:start[cell + 1]]
    for c in range(ncell):
        seg = items[start[c]:start[c + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)


def test_quad_layout_round_trip(gi):
    rng = np.random.default_rng(0)
    for N, C_ in ((8, 3), (16, 2)):
        t = rng.random((5, (N + 2) ** 2, C_)).astype(np.float32)
        q = gi.tiles_to_quads(t, N)
        assert q.shape == (5, (N + 1) ** 2, 4 * C_)
        assert np.array_equal(gi.quads_to_tiles(q, N, C_), t)
        # record (cx, cy) corner 3 is padded texel (cx+1, cy+1)
        T = t.reshape(5, N + 2, N + 2, C_)
        assert np.array_equal(q.reshape(5, N + 1, N + 1, 4, C_)[:, 2, 5, 3], T[:, 3, 6])


def test_empty_image_and_batch_are_no_ops(gi):
    """Width 0 (or n = 0) with otherwise valid arguments returns GI_OK after the
    checks and launches nothing (no device is touched: this runs without one)."""
    lib = gi.load()
    s = gi.GiScene()
    cam = gi.GiCamera()
    cam.width, cam.height = 0, 4
    def gbuf(base):
        g = gi.GiGBuffer()
        g.width, g.height = 0, 4
        g.pos_depth, g.nrm_prim, g.albedo, g.emit = base, base + 16, base + 32, base + 48
        return g
    def res(base):
        r = gi.GiReservoirs()
        r.width, r.height = 0, 4
        r.y_W, r.n_wsum, r.L_M, r.tag_prim = base, base + 16, base + 32, base + 48
        return r
    g, gp = gbuf(1 << 12), gbuf(2 << 12)
    r0, r1, r2 = res(3 << 12), res(4 << 12), res(5 << 12)
    pr = gi.GiProbes()
    pr.dims = (C.c_uint32 * 3)(2, 2, 2)
    pr.irr_res, pr.dep_res = 8, 16
    pr.spacing = gi.F3(1.0, 1.0, 1.0)
    pr.irr, pr.dep = 6 << 12, 7 << 12
    pp = gi.GiParams()
    pp.M, pp.k, pp.radius, pp.g_max, pp.m_cap, pp.depth_rel, pp.subsample = 8, 2, 4.0, 1.0, 20.0, 0.1, 1
    buf = C.c_void_p(8 << 12)
    ok = 0
    assert lib.gi_trace_gbuffer(C.byref(s), C.byref(cam), C.byref(g), None) == ok
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r0),
                                   buf, 1, 0, None) == ok
    assert lib.gi_resample_temporal(C.byref(s), C.byref(g), C.byref(gp), C.byref(cam), C.byref(r0),
                                    C.byref(r1), C.byref(pp), C.byref(r2), 1, 0, None) == ok
    assert lib.gi_resample_spatial(C.byref(s), C.byref(g), C.byref(r0), C.byref(pp), 0, C.byref(r1),
                                   1, 0, None) == ok
    assert lib.gi_shade(C.byref(s), C.byref(g), C.byref(pr), C.byref(r0), buf, C.byref(pp),
                        C.c_void_p(9 << 12), 1, 0, None) == ok
    assert lib.gi_probe_query(C.byref(pr), 0, buf, buf, C.c_void_p(9 << 12), None) == ok
    assert lib.gi_philox(1, 0, buf, C.c_void_p(9 << 12), None) == ok
    assert lib.gi_trace_rays(C.byref(s), 0, buf, buf, C.c_void_p(9 << 12), C.c_void_p(10 << 12), None) == ok


def test_probe_volume_limit(gi):
    """464,000 probes are accepted (the depth records stay under 4 GiB); one
    more is refused before anything runs."""
    lib = gi.load()
    pr = gi.GiProbes()
    pr.irr_res, pr.dep_res = 8, 16
    pr.spacing = gi.F3(1.0, 1.0, 1.0)
    pr.irr, pr.dep = 1 << 12, 2 << 12
    buf = C.c_void_p(3 << 12)
    pr.dims = (C.c_uint32 * 3)(80, 58, 100)
    assert lib.gi_probe_query(C.byref(pr), 0, buf, buf, buf, None) == 0
    pr.dims = (C.c_uint32 * 3)(3, 154667, 1)          # 464,001 probes
    assert lib.gi_probe_query(C.byref(pr), 0, buf, buf, buf, None) == 2
    pr.texel = 1                                      # the same limit for binary16 volumes
    assert lib.gi_probe_query(C.byref(pr), 0, buf, buf, buf, None) == 2
    pr.dims = (C.c_uint32 * 3)(80, 58, 100)
    assert lib.gi_probe_query(C.byref(pr), 0, buf, buf, buf, None) == 0


def test_image_size_limit_of_the_initial_pass(gi):
    """Both forms of the initial pass refuse images of more than 2^23 pixels
    (the reservoir tag holds a 23-bit origin pixel) before anything runs."""
    lib = gi.load()
    s = gi.GiScene()
    W, H = 4097, 2048                               # 2^23 + 2048 pixels
    g = gi.GiGBuffer()
    g.width, g.height = W, H
    g.pos_depth, g.nrm_prim, g.albedo, g.emit = 1 << 12, 2 << 12, 3 << 12, 4 << 12
    r = gi.GiReservoirs()
    r.width, r.height = W, H
    r.y_W, r.n_wsum, r.L_M, r.tag_prim = 5 << 12, 6 << 12, 7 << 12, 8 << 12
    pr = gi.GiProbes()
    pr.dims = (C.c_uint32 * 3)(2, 2, 2)
    pr.irr_res, pr.dep_res = 8, 16
    pr.spacing = gi.F3(1.0, 1.0, 1.0)
    pr.irr, pr.dep = 9 << 12, 10 << 12
    pp = gi.GiParams()
    pp.M, pp.k, pp.radius, pp.g_max, pp.m_cap, pp.depth_rel, pp.subsample = 1, 2, 4.0, 1.0, 20.0, 0.1, 1
    resid = C.c_void_p(11 << 12)
    assert lib.gi_resample_initial(C.byref(s), C.byref(g), C.byref(pr), C.byref(pp), C.byref(r),
                                   resid, 1, 0, None) == 2
    m = gi.GiMlp()
    m.params, m.adam_m, m.adam_v, m.weights, m.scales, m.state = [(12 + i) << 12 for i in range(6)]
    m.pos_lo, m.pos_hi = gi.F3(0.0, 0.0, 0.0), gi.F3(1.0, 1.0, 1.0)
    m.max_rel_err, m.ema_decay = 0.5, 0.0
    ws = C.c_void_p(20 << 12)
    assert lib.gi_resample_initial_mlp(C.byref(s), C.byref(g), C.byref(pr), C.byref(m), C.byref(pp),
                                       C.byref(r), resid, ws, 1 << 40, 1, 0, None) == 2
