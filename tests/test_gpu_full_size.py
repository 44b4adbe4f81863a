"""Every pass at the workloads' full sizes (1920x1080 and 3840x2160), in the
launch configuration the benchmark times, checked on sampled outputs the
oracle computes one by one.

Each pass runs over the whole frame on the device; at the sampled pixels,
and at every pixel their outputs read (spatial neighbours drawn from the
pass's own counters, the temporal reprojection), the inputs are overwritten
with records the oracle computed, so the compared outputs depend on oracle
inputs only.  Probe textures are seeded random stand-ins (the 4K volume has
65,536 probes, too many for the brute-force oracle to fill); the probe
update is checked on sampled probes, from zero textures and from random
textures at hysteresis 0.97.
"""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle as o
from paper_2108_05263_amd import scenegen as sg

from helpers import compare_reservoirs, rel_err

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


def _frozen(cfg):
    """The workload with its probe volume frozen (the textures are inputs here)."""
    return dataclasses.replace(cfg, probe_update=dataclasses.replace(cfg.probe_update, per_frame=False))


@pytest.mark.parametrize("name", ["hd", "uhd"])
def test_passes_full_size_sampled(gi, name):
    cfg = sg.CONFIGS[name]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = sg.random_probe_textures(grid, 11)
    W, H = cfg.width, cfg.height
    pr = cfg.params
    log(f"{name}: device frames 0-1")
    r = gi.Renderer(_frozen(cfg), seed=1, scene=sc)
    r.probe.load(irr, dep)
    r.frame(0)
    r.frame(1)
    torch.cuda.synchronize()
    cam0, cam1 = sg.make_camera(cfg, 0), sg.make_camera(cfg, 1)
    gb1, gb0 = r.gb[1], r.gb[0]

    rng = np.random.default_rng(5)
    S = np.sort(rng.choice(W * H, 2000, replace=False))
    # pixels the spatial passes at S read, from the passes' own counters
    neigh = {int(o.spatial_candidate(W, H, p, j, pr.radius, 1, 1, s))
             for p in S for s in range(pr.n_spatial) for j in range(pr.k)}
    need = np.array(sorted(set(S.tolist()) | (neigh - {-1})), np.int64)
    log(f"{name}: oracle G-buffer + initial on {len(need)} pixels")
    n = W * H
    ogb1 = o.gbuffer(sc, cam1, pixels=need, out=np.zeros((n, 14)))
    # the device's own G-buffer agrees at S before anything is overwritten
    g = gb1.to_records()[S]
    assert np.mean(g[:, 13] == ogb1[S, 13]) > 0.995
    hit = (g[:, 13] == ogb1[S, 13]) & (ogb1[S, 13] != o.MISS)
    e = rel_err(g[hit, 0:3], ogb1[S][hit, 0:3])
    assert np.mean(e) < 1e-5
    ores, oresid = o.resample_initial(sc, W, H, ogb1, grid, irr, dep, pr, 1, 1, pixels=need)
    # previous frame: the reprojected pixels, with initial reservoirs as history
    prev = []
    for p in S:
        if ogb1[p, 13] != o.MISS:
            q = o.reproject(cam0, ogb1[p, 0:3])
            if q >= 0:
                prev.append(q)
    prev = np.array(sorted(set(prev)), np.int64)
    ogb0 = o.gbuffer(sc, cam0, pixels=prev, out=np.zeros((n, 14)))
    ohist, _ = o.resample_initial(sc, W, H, ogb0, grid, irr, dep, pr, 1, 0, pixels=prev)
    active = (ogb1[S, 13] != o.MISS) & (ogb1[S, 6:9].max(1) > 0)

    gb1.load_records(ogb1[need], need)
    gb0.load_records(ogb0[prev], prev)
    rin, rhist, rout = gi.Reservoirs(W, H), gi.Reservoirs(W, H), gi.Reservoirs(W, H)
    resid = torch.zeros(n, 4, device="cuda")
    img = torch.zeros(n, 4, device="cuda")
    tol_flip = 1e-3
    # initial
    gi.resample_initial(r.dscene, gb1, r.probe, pr, rin, resid, 1, 1)
    st, _ = compare_reservoirs(rin.to_records()[S], ores[S], active, tol_flip=tol_flip, label=f"{name} initial")
    er = rel_err(resid.cpu().numpy()[S, :3], oresid[S])
    log(f"{name} initial: {st}; resid {er.mean():.2e}")
    assert er.mean() < 1e-4
    # temporal (current = the oracle's initial reservoirs, history = its previous-frame ones)
    rin.load_records(ores[need], need)
    rhist.load_records(ohist[prev], prev)
    gi.resample_temporal(r.dscene, gb1, gb0, cam0, rin, rhist, pr, rout, 1, 1)
    otmp = o.resample_temporal(sc, W, H, ogb1, ogb0, cam0, ores, ohist, pr, 1, 1, pixels=S)
    st, _ = compare_reservoirs(rout.to_records()[S], otmp[S], active, tol_flip=tol_flip, label=f"{name} temporal")
    log(f"{name} temporal: {st}")
    # spatial passes on the oracle's initial reservoirs
    for s in range(pr.n_spatial):
        gi.resample_spatial(r.dscene, gb1, rin, pr, s, rout, 1, 1)
        osp = o.resample_spatial(sc, W, H, ogb1, ores, pr, s, 1, 1, pixels=S)
        st, _ = compare_reservoirs(rout.to_records()[S], osp[S], active, tol_flip=tol_flip,
                                   label=f"{name} spatial{s}")
        log(f"{name} spatial{s}: {st}")
    # shading of the oracle's initial reservoirs
    resid[torch.as_tensor(S, device="cuda")] = torch.from_numpy(
        np.concatenate([oresid[S], np.zeros((len(S), 1))], 1).astype(np.float32)).cuda()
    gi.shade(r.dscene, gb1, r.probe, rin, resid, pr, img)
    oimg = o.shade(sc, W, H, ogb1, grid, irr, dep, ores, oresid, pr, pixels=S)
    e = rel_err(img.cpu().numpy()[S, :3], oimg[S], 1e-2)
    log(f"{name} shade: mean rel err {e.mean():.2e} max {e.max():.2e}")
    assert e.mean() < 1e-4


@pytest.mark.parametrize("texel", ["f32", "f16"])
def test_probe_update_uhd_sampled(gi, texel):
    """The 4K probe volume (64x16x64 probes, 256 rays, 1024 primitives on the
    grid): a fill pass from zero textures, then a per-frame update at
    hysteresis 0.97 from random textures, and the same update with the
    distance heuristic of Sec. 3.2 (slider 0.8), checked on 64 sampled probes
    (FP32 and binary16 texels)."""
    cfg = dataclasses.replace(sg.CONFIGS["uhd"], probe_texel=texel)
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    u = cfg.probe_update
    ds = gi.DeviceScene(sc, cfg.grid_res)
    pin, pout = gi.Probes(grid), gi.Probes(grid)
    sel = np.sort(np.random.default_rng(6).choice(grid.count, 64, replace=False))
    z_irr, z_dep = sg.empty_probe_textures(grid)
    r_irr, r_dep = sg.random_probe_textures(grid, 7)
    for label, (irr, dep), hyst, frame, slider in (
            ("fill from zero", (z_irr, z_dep), 0.0, gi.FILL_FRAME_BASE, 0.0),
            ("update h=0.97", (r_irr, r_dep), u.hysteresis, 3, 0.0),
            ("update h=0.97, distance slider 0.8", (r_irr, r_dep), u.hysteresis, 4, 0.8)):
        pin.load(irr, dep)
        gi.probe_update(ds, pin, pout, u.rays, hyst, u.sharpness, 1, frame, slider=slider)
        gi_irr, gi_dep = pout.tiles()
        oi, od = o.probe_update(sc, grid, irr[..., :3], dep, u.rays, hyst, u.sharpness, 1, frame, probes=sel,
                                slider=slider)
        ei, ed = rel_err(gi_irr[sel], oi[sel]), rel_err(gi_dep[sel], od[sel])
        log(f"uhd probe update ({texel}, {label}): irr mean {ei.mean():.2e} max {ei.max():.2e}; "
            f"dep mean {ed.mean():.2e} max {ed.max():.2e}")
        assert ei.mean() < 1e-4 and ed.mean() < 1e-4
        assert np.mean(ei > 1e-2) < 1e-3 and np.mean(ed > 1e-2) < 1e-3


def test_probe_query_at_the_volume_limit(gi):
    """The largest probe volume the library accepts, 464,000 probes
    (80 x 58 x 100): its depth records end 3.9 MB short of 4 GiB, the reach
    of the query's 32-bit byte offsets.  Queries in the first and the last
    cells, and anywhere in between, agree with the oracle."""
    grid = sg.probe_grid((80, 58, 100), (0.0, 0.0, 0.0), 1.0)
    assert grid.count == 464000
    irr, dep = sg.random_probe_textures(grid, 9)
    pr = gi.Probes(grid)
    pr.load(irr, dep)
    ext = np.array([80.0, 58.0, 100.0])
    rng = np.random.default_rng(10)
    p = np.concatenate([rng.uniform(0.5, 1.5, (100, 3)), ext - rng.uniform(0.5, 1.5, (100, 3)),
                        rng.uniform(0.0, 1.0, (200, 3)) * ext]).astype(np.float32)
    n = rng.normal(size=(400, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    q = gi.probe_query(pr, torch.from_numpy(p).cuda(), torch.from_numpy(n).cuda()).cpu().numpy()
    del pr
    torch.cuda.empty_cache()
    ref = o.probe_query(grid, irr, dep, p, n)
    e = rel_err(q, ref)
    log(f"464,000 probes: mean rel err {e.mean():.2e} max {e.max():.2e} (last cell {e[100:200].max():.2e})")
    assert e.mean() < 1e-5 and e.max() < 1e-3
