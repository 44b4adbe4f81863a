"""GPU parity of every entry point against the FP64 oracle (through the C ABI).

Shared-input tests feed each kernel the oracle's own inputs for that pass
(oracle G-buffer, probe textures and reservoirs, rounded to float32) so the
comparison isolates the kernel.  Free-running tests let each side run its
own chain.  Tolerances: bit-exact for Philox, tags, M and primitive ids;
relative error (floor 1e-3) of the float fields <= 1e-4 on average over
pixels whose selection agrees; selection flips <= 1e-3 of pixels.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle as o
from paper_2108_05263_amd import scenegen as sg

from helpers import compare_images, compare_reservoirs, rel_err, tags

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gi():
    from paper_2108_05263_amd import gi as m
    m.load()
    assert torch.cuda.is_available()
    return m


# --------------------------------------------------------------------------
# shared fixtures
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny():
    cfg = sg.CONFIGS["tiny"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    return cfg, sc, grid, irr, dep


@pytest.fixture(scope="module")
def hd_small():
    """The 1080p room at 250x141 (ragged tiles), probes filled by the oracle
    with fewer rays (the textures are an input of the resampling passes)."""
    cfg = sg.CONFIGS["hd"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    upd = sg.ProbeUpdate(rays=32, fill_passes=2, fill_rays=32)
    irr, dep = o.fill_probes(sc, grid, upd, seed=1)
    return cfg, sc, grid, irr, dep


def _setup(gi, sc, grid, irr, dep, W, H, use_grid):
    cfg_grid = (32, 8, 32) if sc.n_prims > 16 else (8, 8, 8)
    ds = gi.DeviceScene(sc, cfg_grid if use_grid else None)
    pr = gi.Probes(grid)
    pr.load(irr, dep)
    return ds, pr


# --------------------------------------------------------------------------
# Philox and the tracer
# --------------------------------------------------------------------------
def test_philox_bit_exact(gi):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, (3000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [2073599, 7, 0, 31], [5, 0xF0000003, 9, 255]]
    for seed in (1, 0x0123456789ABCDEF):
        out = gi.philox(seed, torch.from_numpy(ctr.view(np.int32)).cuda()).cpu().numpy().view(np.uint32)
        ref = np.array([o.philox(seed, c) for c in ctr])
        assert np.array_equal(out, ref)


@pytest.mark.parametrize("name", ["tiny", "hd"])
def test_tracer_matches_oracle_and_grid_matches_brute(gi, name):
    cfg = sg.CONFIGS[name]
    sc = sg.make_scene(cfg)
    rng = np.random.default_rng(1)
    lo, hi = sc.room_lo.astype(np.float64), sc.room_hi.astype(np.float64)
    org = rng.uniform(lo + 0.05, hi - 0.05, (4000, 3)).astype(np.float32)
    log(f"tracer {name}: {len(org)} rays")
    d = rng.normal(size=(4000, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    og, dg = torch.from_numpy(org).cuda(), torch.from_numpy(d).cuda()
    brute = gi.DeviceScene(sc)
    grid = gi.DeviceScene(sc, cfg.grid_res)
    ob, pb = gi.trace_rays(brute, og, dg)
    ogr, pgr = gi.trace_rays(grid, og, dg)
    ob, pb, ogr, pgr = ob.cpu().numpy(), pb.cpu().numpy(), ogr.cpu().numpy(), pgr.cpu().numpy()
    # grid walk returns exactly the brute-force hit
    bad = np.where((pb != pgr) | np.any(ob != ogr, axis=1))[0]
    for i in bad[:5]:
        log(f"grid/brute mismatch {i}: org {org[i]} d {d[i]} brute {ob[i]} {pb[i]} grid {ogr[i]} {pgr[i]}")
    assert len(bad) == 0, f"{len(bad)} grid/brute mismatches"
    ref = [o.closest_hit(sc, org[i].astype(np.float64), d[i].astype(np.float64)) for i in range(len(org))]
    prim_ref = np.array([r[2] for r in ref], np.int64)
    t_ref = np.array([r[1] for r in ref])
    n_ref = np.array([r[3] for r in ref])
    same = pb.astype(np.int64) & 0xFFFFFFFF == prim_ref
    log(f"tracer {name}: prim agreement {same.mean():.5f}")
    assert same.mean() >= 0.999
    # FP32 hit distances: the root of a near-tangent ray is ill-conditioned,
    # so the bound is on the mean and on the tail fraction
    et = rel_err(ob[same, 0], t_ref[same], 1e-3)
    log(f"tracer {name}: t rel err mean {et.mean():.2e} max {et.max():.2e}")
    assert et.mean() < 1e-6 and np.mean(et > 1e-4) <= 1e-3 and et.max() < 1e-2
    en = np.abs(ob[same, 1:4] - n_ref[same]).max(1)
    assert np.mean(en > 1e-4) <= 1e-3 and en.max() < 1e-2


# --------------------------------------------------------------------------
# G-buffer, probe query, probe update
# --------------------------------------------------------------------------
@pytest.mark.parametrize("W,H", [(64, 64), (250, 141)])
def test_gbuffer(gi, W, H):
    cfg = sg.CONFIGS["tiny" if W == 64 else "hd"]
    sc = sg.make_scene(cfg)
    cam = sg.make_camera(cfg, 0, W, H)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    gb = gi.GBuffer(W, H)
    gi.trace_gbuffer(ds, cam, gb)
    g = gb.to_records()
    r = o.gbuffer(sc, cam)
    same = g[:, 13] == r[:, 13]
    log(f"gbuffer {W}x{H}: prim agreement {same.mean():.6f}")
    assert same.mean() >= 0.999
    assert np.max(np.abs(g[same, 0:3] - r[same, 0:3])) < 1e-4
    assert np.max(np.abs(g[same, 3:6] - r[same, 3:6])) < 1e-4
    assert np.array_equal(g[same, 6:12], r[same, 6:12].astype(np.float32).astype(np.float64))
    assert np.max(rel_err(g[same, 12], r[same, 12])) < 1e-5


TEXELS = pytest.mark.parametrize("texel", ["f32", "f16"])


@TEXELS
def test_probe_query(gi, tiny, texel):
    cfg, sc, grid, irr, dep = tiny
    grid = dataclasses.replace(grid, texel=texel)
    pr = gi.Probes(grid)
    pr.load(irr, dep)
    rng = np.random.default_rng(2)
    p = rng.uniform(0.0, 8.0, (5000, 3)).astype(np.float32)
    n = rng.normal(size=(5000, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    q = gi.probe_query(pr, torch.from_numpy(p).cuda(), torch.from_numpy(n).cuda()).cpu().numpy()
    ref = o.probe_query(grid, irr.astype(np.float32), dep.astype(np.float32), p, n)
    e = rel_err(q, ref)
    log(f"probe query ({texel}): mean rel err {e.mean():.2e} max {e.max():.2e}")
    assert e.mean() < 1e-5 and e.max() < 1e-3


@TEXELS
def test_probe_layout_odd_volume(gi, tiny, texel):
    """A 3x5x2 probe volume (no power-of-two extent, P = 30): the query on
    points inside and around it, and the probe update's read-back, agree with
    the oracle, which indexes probe-major tiles, through the library's
    quad-major irradiance records."""
    cfg, sc, _, _, _ = tiny
    grid = sg.probe_grid((3, 5, 2), (0.5, 0.25, 1.0), 1.5, texel=texel)   # inside the 8-unit room
    irr, dep = sg.random_probe_textures(grid, 5)
    pr = gi.Probes(grid)
    pr.load(irr, dep)
    ti, td = pr.tiles()
    if texel == "f16":
        # texels come back at binary16: irradiance, and depth as (mean, variance)
        assert np.array_equal(ti, irr[..., :3].astype(np.float16).astype(np.float32))
        d = dep[..., :2].astype(np.float64)
        mu = d[..., 0].astype(np.float16).astype(np.float64)
        var = (d[..., 1] - d[..., 0] * d[..., 0]).astype(np.float16).astype(np.float64)
        assert np.array_equal(td[..., 0], mu) and np.array_equal(td[..., 1], var + mu * mu)
    else:
        # FP32 texels come back as loaded
        assert np.array_equal(ti, irr[..., :3].astype(np.float32))
        assert np.array_equal(td, dep[..., :2].astype(np.float32).astype(np.float64))
    rng = np.random.default_rng(4)
    p = rng.uniform(-0.5, 8.0, (4000, 3)).astype(np.float32)
    n = rng.normal(size=(4000, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    q = gi.probe_query(pr, torch.from_numpy(p).cuda(), torch.from_numpy(n).cuda()).cpu().numpy()
    ref = o.probe_query(grid, irr.astype(np.float32), dep.astype(np.float32), p, n)
    e = rel_err(q, ref)
    log(f"odd volume query ({texel}): mean rel err {e.mean():.2e} max {e.max():.2e}")
    assert e.mean() < 1e-5 and e.max() < 1e-3
    ds = gi.DeviceScene(sc, cfg.grid_res)
    pout = gi.Probes(grid)
    gi.probe_update(ds, pr, pout, 64, 0.5, 50.0, 1, 7)
    gi_irr, gi_dep = pout.tiles()
    assert np.array_equal(pout.irr_quads(), gi.tiles_to_quads(gi_irr, grid.irr_res))
    ri, rd = o.probe_update(sc, grid, irr.astype(np.float32), dep.astype(np.float32), 64, 0.5, 50.0, 1, 7)
    ei, ed = rel_err(gi_irr, ri), rel_err(gi_dep, rd)
    log(f"odd volume update ({texel}): irr mean {ei.mean():.2e}; dep mean {ed.mean():.2e}")
    assert ei.mean() < 1e-4 and ed.mean() < 1e-4


@TEXELS
def test_probe_update(gi, tiny, texel):
    cfg, sc, grid, irr, dep = tiny
    # start from the third fill pass so the recursion's Q_prev is non-trivial
    i2, d2 = o.fill_probes(sc, grid, sg.ProbeUpdate(fill_passes=2, fill_rays=64), seed=1)
    i2, d2 = i2.astype(np.float32), d2.astype(np.float32)
    grid = dataclasses.replace(grid, texel=texel)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    pin, pout = gi.Probes(grid), gi.Probes(grid)
    pin.load(i2, d2)
    for hyst, slider in ((0.0, 0.0), (0.97, 0.0), (0.0, 0.8)):
        gi.probe_update(ds, pin, pout, 64, hyst, 50.0, 1, 5, slider=slider)
        gi_irr, gi_dep = pout.tiles()
        # every quad record agrees with the padded tile it encodes (gutters included)
        assert np.array_equal(pout.irr_quads(), gi.tiles_to_quads(gi_irr, grid.irr_res))
        assert np.array_equal(pout.dep_quads(), gi.tiles_to_quads(gi_dep, grid.dep_res))
        ri, rd = o.probe_update(sc, grid, i2, d2, 64, hyst, 50.0, 1, 5, slider=slider)
        ei, ed = rel_err(gi_irr, ri), rel_err(gi_dep, rd)
        log(f"probe update ({texel}) h={hyst} slider={slider}: irr mean {ei.mean():.2e} max {ei.max():.2e}; "
            f"dep mean {ed.mean():.2e} max {ed.max():.2e}")
        assert ei.mean() < 1e-4 and ed.mean() < 1e-4
        assert np.mean(ei > 1e-2) < 1e-3 and np.mean(ed > 1e-2) < 1e-3


# --------------------------------------------------------------------------
# resampling passes with shared inputs
# --------------------------------------------------------------------------
def _pass_inputs(sc, grid, irr, dep, cfg, W, H, frames=2):
    """Oracle chain over `frames` frames; returns per-frame stage records."""
    seq = o.Sequence(sc, grid, irr, dep, cfg.params, 1)
    out = []
    for f in range(frames):
        cam = sg.make_camera(cfg, f, W, H)
        img, st = seq.frame(cam, f)
        st["cam"] = cam
        out.append(st)
    return out


def _check_chain(gi, cfg, sc, grid, irr, dep, W, H, frames, which):
    """Each pass of the last of `frames` oracle frames, run on the GPU on the
    oracle's own inputs (G-buffer, reservoirs, residual) and compared."""
    st = _pass_inputs(sc, grid, irr, dep, cfg, W, H, frames)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    pr = cfg.params
    gb, gbp = gi.GBuffer(W, H), gi.GBuffer(W, H)
    rin, rin2, rout = gi.Reservoirs(W, H), gi.Reservoirs(W, H), gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    img = torch.zeros(W * H, 4, device="cuda")
    f = frames - 1
    s = st[f]
    gb.load_records(s["gbuffer"])
    active = (s["gbuffer"][:, 13] != o.MISS) & (s["gbuffer"][:, 6:9].max(1) > 0)
    # initial
    gi.resample_initial(ds, gb, probes, pr, rout, resid, 1, f)
    res, _ = compare_reservoirs(rout.to_records(), s["initial"], active, label=f"{which} initial")
    er = rel_err(resid.cpu().numpy()[:, :3], s["resid"])
    log(f"{which} initial: {res}; resid mean {er.mean():.2e}")
    assert er.mean() < 1e-4
    dev_resid = resid.cpu().numpy()[:, :3].copy()
    # temporal
    if "temporal" in s:
        gbp.load_records(st[f - 1]["gbuffer"])
        rin.load_records(s["initial"])
        rin2.load_records(st[f - 1][f"spatial{pr.n_spatial - 1}"])
        gi.resample_temporal(ds, gb, gbp, st[f - 1]["cam"], rin, rin2, pr, rout, 1, f)
        res, _ = compare_reservoirs(rout.to_records(), s["temporal"], active, label=f"{which} temporal")
        log(f"{which} temporal: {res}")
    # spatial passes
    src = s["temporal"] if "temporal" in s else s["initial"]
    for sp in range(pr.n_spatial):
        rin.load_records(src)
        gi.resample_spatial(ds, gb, rin, pr, sp, rout, 1, f)
        res, _ = compare_reservoirs(rout.to_records(), s[f"spatial{sp}"], active,
                                    label=f"{which} spatial{sp}")
        log(f"{which} spatial{sp}: {res}")
        src = s[f"spatial{sp}"]
    # shade
    rin.load_records(src)
    resid.copy_(torch.from_numpy(np.concatenate([s["resid"], np.zeros((W * H, 1))], 1).astype(np.float32)))
    gi.shade(ds, gb, probes, rin, resid, pr, img)
    gimg = img.cpu().numpy()[:, :3]
    e = rel_err(gimg, s["image"], 1e-2)
    log(f"{which} shade: mean rel err {e.mean():.2e} max {e.max():.2e}")
    assert e.mean() < 1e-4
    return dev_resid, s["resid"]


@pytest.mark.parametrize("which,texel", [("tiny", "f32"), ("hd_small", "f32"), ("tiny", "f16"), ("hd_small", "f16")])
def test_passes_shared_inputs(gi, request, which, texel):
    """Every pass on the oracle's inputs, with the FP32 probe volume of the
    workloads and with a binary16 one (each side reading the textures at that
    precision)."""
    cfg, sc, grid, irr, dep = request.getfixturevalue(which)
    grid = dataclasses.replace(grid, texel=texel)
    W, H = (64, 64) if which == "tiny" else (250, 141)
    _check_chain(gi, cfg, sc, grid, irr, dep, W, H, 1 if which == "tiny" else 2, f"{which} {texel}")


@pytest.mark.parametrize("variant", ["biased", "no_bound", "tight_bound", "subsample", "fractional_cap"])
def test_chain_parameter_variants(gi, tiny, variant):
    """The chain over two frames (initial, temporal, two spatial passes,
    shading) on shared inputs with the biased 1/M normalisation, with a G_max
    no geometry term reaches (nothing bounded, the residual exactly zero), with
    a tight G_max = 0.05 (the residual nonzero at six times as many pixels),
    with candidate subsampling (half the pixels draw nothing in frame 1 and
    take over their history) and with a history cap of 2.3 x M (rounded down)."""
    cfg, sc, grid, irr, dep = tiny
    over = {"biased": dict(unbiased=0), "no_bound": dict(g_max=1e30), "tight_bound": dict(g_max=0.05),
            "subsample": dict(subsample=2), "fractional_cap": dict(m_cap=2.3)}[variant]
    cfg = dataclasses.replace(cfg, params=dataclasses.replace(cfg.params, temporal=True, n_spatial=2, **over))
    resid, oresid = _check_chain(gi, cfg, sc, grid, irr, dep, 64, 64, 2, f"tiny {variant}")
    if variant == "no_bound":
        assert np.all(resid == 0.0) and np.all(oresid == 0.0)
    if variant == "tight_bound":
        assert np.mean(oresid.max(1) > 0) > 0.2  # about 5% at the default G_max = 1


# --------------------------------------------------------------------------
# free-running
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which,frames", [("tiny", 1), ("hd_small", 3)])
def test_free_running(gi, request, which, frames):
    cfg, sc, grid, irr, dep = request.getfixturevalue(which)
    W, H = (64, 64) if which == "tiny" else (250, 141)
    r = gi.Renderer(cfg, seed=1, width=W, height=H, scene=sc)
    r.probe.load(irr, dep)
    seq = o.Sequence(sc, grid, irr, dep, cfg.params, 1)
    for f in range(frames):
        hist = r.frame(f)
        oimg, st = seq.frame(sg.make_camera(cfg, f, W, H), f)
        torch.cuda.synchronize()
        fin = st[f"spatial{cfg.params.n_spatial - 1}"]
        g = hist.to_records()
        same = (tags(g) == tags(fin))
        active = (st["gbuffer"][:, 13] != o.MISS) & (st["gbuffer"][:, 6:9].max(1) > 0)
        flips = float(np.mean(~same[active]))
        gimg = r.img.cpu().numpy()[:, :3]
        m = compare_images(gimg, oimg, same, tol=1e-4, label=f"{which} frame {f}")
        log(f"free-running {which} frame {f}: flips {flips:.2e}, mean rel image err (unflipped) {m:.2e}")
        assert flips <= 1e-3


def _lds_vs_global(gi, cfg, sc, irr, dep, W, H):
    out = []
    for lds in (True, False):
        r = gi.Renderer(cfg, seed=2, width=W, height=H, scene=sc, lds=lds)
        r.probe.load(irr, dep)
        for f in range(2):
            r.frame(f)
        torch.cuda.synchronize()
        out.append((r.img.cpu().numpy().copy(), r.hist.to_records()))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("which", ["tiny", "hd_small"])
def test_lds_staging_matches_global(gi, request, which):
    """Tracing from the LDS copy of the scene gives bit-identical frames."""
    cfg, sc, grid, irr, dep = request.getfixturevalue(which)
    W, H = (64, 64) if which == "tiny" else (250, 141)
    _lds_vs_global(gi, cfg, sc, irr, dep, W, H)


def test_lds_staging_matches_global_interleaved_types(gi, hd_small):
    """The initial pass reorders each staged cell's items (spheres, then
    boxes).  With the room's primitives renumbered in a shuffled order the
    types interleave in id order, so the reordering swaps items in most
    cells; the frames stay bit-identical to the walk over the caller's
    id-ordered lists (the closest hit is the smallest (t, id) pair)."""
    cfg, sc, grid, irr, dep = hd_small
    perm = np.random.default_rng(5).permutation(sc.n_prims)
    sc2 = dataclasses.replace(sc, prims=np.ascontiguousarray(sc.prims[perm]))
    types = sc2.prims.view(np.uint32)[:, 3]
    assert np.sum(np.diff(types.astype(np.int64)) != 0) > sc.n_prims // 4
    log(f"interleaved types: {int(np.sum(np.diff(types.astype(np.int64)) != 0))} type changes in id order")
    _lds_vs_global(gi, cfg, sc2, irr, dep, 250, 141)


def test_determinism(gi, tiny):
    cfg, sc, grid, irr, dep = tiny
    imgs = []
    for _ in range(2):
        r = gi.Renderer(cfg, seed=3, scene=sc)
        r.probe.load(irr, dep)
        r.frame(0)
        torch.cuda.synchronize()
        imgs.append((r.img.cpu().numpy().copy(), r.hist.to_records()))
    assert np.array_equal(imgs[0][0], imgs[1][0])
    assert np.array_equal(imgs[0][1], imgs[1][1])


# --------------------------------------------------------------------------
# full size
# --------------------------------------------------------------------------
def test_furnace_full_hd(gi):
    rho, L = np.array([0.5, 0.7, 0.9], np.float32), np.array([1.0, 2.0, 3.0], np.float32)
    sc = sg.furnace_plane(albedo=rho, sky=L)
    cam = sg.furnace_camera(1920, 1080)
    cfg = sg.CONFIGS["hd"]
    r = gi.Renderer(cfg, seed=5, scene=sc, use_grid=False)
    r.cfg = cfg
    for f in range(2):
        r.frame(f, cam=cam)
    torch.cuda.synchronize()
    img = r.img.cpu().numpy()[:, :3].astype(np.float64)
    gb = r.gb[1].to_records()
    on = gb[:, 13] != o.MISS
    e = rel_err(img[on], rho.astype(np.float64) * L.astype(np.float64), 0.0)
    log(f"furnace 1080p: max rel err {e.max():.2e}")
    assert e.max() < 2e-5
    assert np.array_equal(img[~on], np.broadcast_to(L.astype(np.float64), img[~on].shape))


@pytest.mark.parametrize("M", [1, 32])
def test_initial_candidate_count_extremes(gi, tiny, M):
    """The initial pass with a single candidate (M = 1: the selected sample is
    the candidate, W = 1/p) and with the most the library takes (M =
    GI_MAX_M = 32), on shared inputs."""
    cfg, sc, grid, irr, dep = tiny
    W, H = 64, 64
    pr = dataclasses.replace(cfg.params, M=M)
    ogb = o.gbuffer(sc, sg.make_camera(cfg, 0, W, H))
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    gb = gi.GBuffer(W, H)
    gb.load_records(ogb)
    out = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    gi.resample_initial(ds, gb, probes, pr, out, resid, 1, 0)
    active = (ogb[:, 13] != o.MISS) & (ogb[:, 6:9].max(1) > 0)
    res, _ = compare_reservoirs(out.to_records(), ores, active, label=f"M={M} initial")
    er = rel_err(resid.cpu().numpy()[:, :3], oresid)
    log(f"M={M} initial: {res}; resid mean {er.mean():.2e}")
    assert er.mean() < 1e-4
    assert np.all(out.to_records()[active, 11] == M)


@pytest.mark.parametrize("k", [0, 8])
def test_spatial_neighbour_count_extremes(gi, tiny, k):
    """Spatial reuse with no neighbour (k = 0: the pixel's own reservoir,
    normalised again) and with the most the library takes (k = GI_MAX_K = 8),
    both passes, on shared inputs."""
    cfg, sc, grid, irr, dep = tiny
    W, H = 64, 64
    pr = dataclasses.replace(cfg.params, k=k)
    ogb = o.gbuffer(sc, sg.make_camera(cfg, 0, W, H))
    ores, _ = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    gb = gi.GBuffer(W, H)
    gb.load_records(ogb)
    rin, rout = gi.Reservoirs(W, H), gi.Reservoirs(W, H)
    rin.load_records(ores)
    active = (ogb[:, 13] != o.MISS) & (ogb[:, 6:9].max(1) > 0)
    for sp in range(2):
        gi.resample_spatial(ds, gb, rin, pr, sp, rout, 1, 0)
        osp = o.resample_spatial(sc, W, H, ogb, ores, pr, sp, 1, 0)
        res, _ = compare_reservoirs(rout.to_records(), osp, active, label=f"k={k} spatial{sp}")
        log(f"k={k} spatial{sp}: {res}")


@pytest.mark.parametrize("variant", ["plain", "emitters", "subsample", "binary16"])
def test_initial_full_hd_sampled(gi, variant):
    """The 1920x1080 workload's G-buffer and initial pass in the launch
    configuration the benchmark times, checked on 1500 sampled pixels; also
    with emitter-sampled candidates (M = 28 + 4) and with candidate
    subsampling (n = 2), the options of Sec. 3.1 step 1 and Sec. 6, and
    from binary16 probe textures."""
    cfg = sg.CONFIGS["hd"]
    if variant == "binary16":
        cfg = dataclasses.replace(cfg, probe_texel="f16")
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    upd = sg.ProbeUpdate(rays=32, fill_passes=2, fill_rays=32)
    irr, dep = o.fill_probes(sc, grid, upd, seed=1)
    r = gi.Renderer(cfg, seed=1, scene=sc)
    r.probe.load(irr, dep)
    r.frame(0)
    torch.cuda.synchronize()
    W, H = cfg.width, cfg.height
    rng = np.random.default_rng(4)
    pix = np.sort(rng.choice(W * H, 2000, replace=False))
    cam = sg.make_camera(cfg, 0)
    ogb = o.gbuffer(sc, cam, pixels=pix)
    gb_g = r.gb[0].to_records()
    assert np.mean(gb_g[pix, 13] == ogb[pix, 13]) > 0.999
    # initial reservoirs of the device run are gone (buffers rotate); rerun it
    rr = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    pr = {"plain": cfg.params, "emitters": dataclasses.replace(cfg.params, M=28, M_light=4),
          "subsample": dataclasses.replace(cfg.params, subsample=2), "binary16": cfg.params}[variant]
    gi.resample_initial(r.dscene, r.gb[0], r.probe, pr, rr, resid, 1, 0)
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0, pixels=pix)
    g = rr.to_records()[pix]
    ref = ores[pix]
    active = (ogb[pix, 13] != o.MISS) & (ogb[pix, 6:9].max(1) > 0) & (gb_g[pix, 13] == ogb[pix, 13])
    res, _ = compare_reservoirs(g, ref, active, tol_flip=1e-3, label=f"1080p initial sampled ({variant})")
    er = rel_err(resid.cpu().numpy()[pix, :3], oresid[pix])
    log(f"1080p initial (sampled, {variant}): {res}; resid mean {er.mean():.2e}")
    assert er.mean() < 1e-4


# --------------------------------------------------------------------------
# emitter-sampled candidates
# --------------------------------------------------------------------------
def test_emitter_candidates_shared_inputs(gi, tiny):
    """M cosine + M_light emitter candidates (balance heuristic) on the
    oracle's G-buffer and probes: reservoirs and image against the oracle."""
    cfg, sc, grid, irr, dep = tiny
    W, H = 64, 64
    pr = dataclasses.replace(cfg.params, M=6, M_light=4)
    cam = sg.make_camera(cfg, 0, W, H)
    ogb = o.gbuffer(sc, cam)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    assert ds.c.n_emitters == 1
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    gb = gi.GBuffer(W, H)
    gb.load_records(ogb)
    out = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    gi.resample_initial(ds, gb, probes, pr, out, resid, 1, 0)
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0)
    active = (ogb[:, 13] != o.MISS) & (ogb[:, 6:9].max(1) > 0)
    st, _ = compare_reservoirs(out.to_records(), ores, active, label="emitter candidates")
    assert np.all(out.to_records()[active, 11] == 10)
    # some reservoirs hold an emitter sample drawn by light sampling (candidate index >= M)
    cand = (tags(ores[active]) >> 4) & 31
    assert np.mean(cand >= 6) > 0.05
    er = rel_err(resid.cpu().numpy()[:, :3], oresid)
    log(f"emitter candidates: {st}; resid {er.mean():.2e}")
    assert er.mean() < 1e-4
    img = torch.zeros(W * H, 4, device="cuda")
    gi.shade(ds, gb, probes, out, resid, pr, img)
    oimg = o.shade(sc, W, H, ogb, grid, irr, dep, ores, oresid, pr)
    e = rel_err(img.cpu().numpy()[:, :3], oimg, 1e-2)
    log(f"emitter candidates shade: mean rel err {e.mean():.2e}")
    assert e.mean() < 1e-4


def test_emitter_candidates_closed_form(gi):
    """The two-sphere closed form of the oracle's pin, on the device: each
    plane pixel's mean over seeds is rho sum_e L_e (r_e/d_e)^2 cos(theta_e)."""
    sys.path.insert(0, __import__("os").path.dirname(__file__))
    from test_oracle_resampling import _sphere_over_plane
    sc, cam, rho, Le, r, c = _sphere_over_plane()
    W, H = cam.width, cam.height
    ogb = o.gbuffer(sc, cam)
    plane = (ogb[:, 13] == 0) & (np.abs(ogb[:, 4] - 1.0) < 1e-12)
    x = ogb[plane, 0:3]
    exact = np.zeros((len(x), 3))
    for e in range(2):
        v = c[e] - x
        d = np.linalg.norm(v, axis=1)
        exact += rho[None, :] * Le[e][None, :] * ((r[e] / d) ** 2 * (v[:, 1] / d))[:, None]
    grid = sg.probe_grid((2, 2, 2), (-8.0, -1.0, -8.0), 8.0)
    ds = gi.DeviceScene(sc, None)
    probes = gi.Probes(grid)
    gb = gi.GBuffer(W, H)
    gb.load_records(ogb)
    pr = sg.Params(M=2, M_light=8, k=0, n_spatial=0, temporal=False)
    out = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    img = torch.zeros(W * H, 4, device="cuda")
    S = 400
    vals = np.zeros((S, int(plane.sum()), 3))
    for s in range(S):
        gi.resample_initial(ds, gb, probes, pr, out, resid, 2000 + s, 0)
        gi.shade(ds, gb, probes, out, resid, pr, img)
        vals[s] = img.cpu().numpy()[plane, :3]
    mean, sd = vals.mean(0), vals.std(0, ddof=1)
    z = (mean - exact) / (sd / np.sqrt(S) + 1e-12)
    log(f"emitter closed form on the device: max |z| {np.abs(z).max():.2f}")
    assert np.abs(z).max() < 5.0


@pytest.mark.parametrize("n", [2, 3])
def test_subsampled_initial_shared_inputs(gi, tiny, n):
    """Candidate subsampling: only pixels on the (x + y + f) % n pattern draw
    candidates; against the oracle on its own G-buffer and probes."""
    cfg, sc, grid, irr, dep = tiny
    W, H = 64, 64
    pr = dataclasses.replace(cfg.params, subsample=n)
    ogb = o.gbuffer(sc, sg.make_camera(cfg, 0, W, H))
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    gb = gi.GBuffer(W, H)
    gb.load_records(ogb)
    out = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    gi.resample_initial(ds, gb, probes, pr, out, resid, 1, 3)
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 3)
    active = (ogb[:, 13] != o.MISS) & (ogb[:, 6:9].max(1) > 0)
    g = out.to_records()
    assert np.array_equal(g[:, 11], ores[:, 11])
    st, _ = compare_reservoirs(g, ores, active, label=f"subsample {n}")
    er = rel_err(resid.cpu().numpy()[:, :3], oresid)
    log(f"subsample {n}: {st}; resid {er.mean():.2e}")
    assert er.mean() < 1e-4


def test_binding_refuses_buffers_of_another_dtype(gi, tiny):
    """The library writes float32 records: a float64 or strided output buffer
    is refused before any launch instead of being misread."""
    cfg, sc, grid, irr, dep = tiny
    W = H = 16
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    g = gi.GBuffer(W, H)
    out = gi.Reservoirs(W, H)
    with pytest.raises(gi.GiError):
        gi.resample_initial(ds, g, probes, cfg.params, out, torch.zeros(W * H, 4, dtype=torch.float64, device="cuda"), 1, 0)
    with pytest.raises(gi.GiError):
        gi.resample_initial(ds, g, probes, cfg.params, out, torch.zeros(W * H, 8, device="cuda")[:, ::2], 1, 0)
