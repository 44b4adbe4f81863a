"""Precision variants (the 4K precision sweep): G-buffer normals and albedo
stored in half precision.

* the half-precision G-buffer against the oracle's G-buffer rounded to
  half (storage emulation: the oracle computes in FP64, only its stored
  normals and albedo are rounded, as the device stores them);
* the passes on shared inputs with that rounding, at the path's usual bar;
* the error each storage format leaves against the unrounded FP64 oracle at
  3840x2160 on sampled pixels (the per-dtype error statement), bounded by
  what half precision's 11 significant bits allow.
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


def _round_half(gb, renormalise=True):
    """Storage emulation: normals and albedo of oracle G-buffer records
    rounded to half precision (nearest even), normals renormalised as the
    device reads them; the rest untouched."""
    r = gb.copy()
    r[:, 3:9] = r[:, 3:9].astype(np.float16).astype(np.float64)
    if renormalise:
        ln = np.linalg.norm(r[:, 3:6], axis=1, keepdims=True)
        r[:, 3:6] = np.where(ln > 0, r[:, 3:6] / np.where(ln > 0, ln, 1.0), 0.0)
    return r


def test_gbuffer_half(gi):
    cfg = sg.CONFIGS["hd"]
    sc = sg.make_scene(cfg)
    W, H = 250, 141
    cam = sg.make_camera(cfg, 0, W, H)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    g = gi.GBuffer(W, H, fmt="f16")
    gi.trace_gbuffer(ds, cam, g)
    got = g.to_records()      # the stored half values (not renormalised)
    ref = _round_half(o.gbuffer(sc, cam), renormalise=False)
    same = got[:, 13] == ref[:, 13]
    assert same.mean() > 0.999
    hit = same & (ref[:, 13] != o.MISS)
    # half of the FP32 value vs half of the FP64 value: equal, or (at a rounding
    # boundary, or where a grazing hit moved) a few half-ulp steps apart
    dn = np.abs(got[hit, 3:9] - ref[hit, 3:9])
    ulp = np.maximum(np.abs(ref[hit, 3:9]), 2.0 ** -14) * 2.0 ** -10
    log(f"half G-buffer: equal {np.mean(dn == 0):.5f}, within one step {np.mean(dn <= ulp * 1.0001):.5f}, "
        f"max {dn.max():.2e}")
    assert np.mean(dn <= ulp * 1.0001) > 0.999
    assert np.mean(dn == 0) > 0.99
    assert np.allclose(got[hit, 0:3], ref[hit, 0:3], rtol=0, atol=1e-4)
    assert np.all(got[~(ref[:, 13] != o.MISS), 13] == o.MISS)


def test_passes_half_gbuffer_shared_inputs(gi):
    """Initial pass and shading on the oracle's G-buffer with half-precision
    normals and albedo (both sides read the same rounded values)."""
    cfg = sg.CONFIGS["tiny"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = o.fill_probes(sc, grid, cfg.probe_update, seed=1)
    W, H = 64, 64
    pr = cfg.params
    ogb = _round_half(o.gbuffer(sc, sg.make_camera(cfg, 0, W, H)))
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    g = gi.GBuffer(W, H, fmt="f16")
    g.load_records(_round_half(o.gbuffer(sc, sg.make_camera(cfg, 0, W, H)), renormalise=False))
    out = gi.Reservoirs(W, H)
    resid = torch.zeros(W * H, 4, device="cuda")
    gi.resample_initial(ds, g, probes, pr, out, resid, 1, 0)
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0)
    active = (ogb[:, 13] != o.MISS) & (ogb[:, 6:9].max(1) > 0)
    st, _ = compare_reservoirs(out.to_records(), ores, active, label="half G-buffer initial")
    img = torch.zeros(W * H, 4, device="cuda")
    gi.shade(ds, g, probes, out, resid, pr, img)
    oimg = o.shade(sc, W, H, ogb, grid, irr, dep, ores, oresid, pr)
    e = rel_err(img.cpu().numpy()[:, :3], oimg, 1e-2)
    log(f"half G-buffer: {st}; image {e.mean():.2e}")
    assert e.mean() < 1e-4


def test_storage_error_uhd_sampled(gi):
    """3840x2160: each format's own chain (G-buffer, initial pass, shading)
    against the FP64 oracle without storage rounding, on 400 sampled pixels.
    FP32 stays at the parity bar; half precision (11 significant bits,
    relative rounding <= 2^-11 in normals and albedo) leaves an image error
    of order 1e-3, bounded here by 1e-2."""
    cfg = sg.CONFIGS["uhd"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = sg.random_probe_textures(grid, 11)
    W, H = cfg.width, cfg.height
    n = W * H
    pr = cfg.params
    cam = sg.make_camera(cfg, 0)
    S = np.sort(np.random.default_rng(8).choice(n, 2000, replace=False))
    ogb = o.gbuffer(sc, cam, pixels=S, out=np.zeros((n, 14)))
    ores, oresid = o.resample_initial(sc, W, H, ogb, grid, irr, dep, pr, 1, 0, pixels=S)
    oimg = o.shade(sc, W, H, ogb, grid, irr, dep, ores, oresid, pr, pixels=S)
    ds = gi.DeviceScene(sc, cfg.grid_res)
    probes = gi.Probes(grid)
    probes.load(irr, dep)
    errs = {}
    for fmt in ("f32", "f16"):
        g = gi.GBuffer(W, H, fmt=fmt)
        gi.trace_gbuffer(ds, cam, g)
        out = gi.Reservoirs(W, H)
        resid = torch.zeros(n, 4, device="cuda")
        img = torch.zeros(n, 4, device="cuda")
        gi.resample_initial(ds, g, probes, pr, out, resid, 1, 0)
        gi.shade(ds, g, probes, out, resid, pr, img)
        gr = g.to_records()[S]
        keep = (gr[:, 13] == ogb[S, 13])
        rr = out.to_records()[S]
        flips = np.mean((rr[:, 12] != ores[S, 12]) & keep & (ogb[S, 13] != o.MISS))
        same = keep & (rr[:, 12] == ores[S, 12])
        e = rel_err(img.cpu().numpy()[S, :3][same], oimg[S][same], 1e-2)
        errs[fmt] = (float(e.mean()), float(flips))
        log(f"uhd {fmt} G-buffer vs FP64 oracle: image mean rel err {e.mean():.2e} (unflipped), "
            f"flips {flips:.2e}")
        del g, out, resid, img
        torch.cuda.empty_cache()
    assert errs["f32"][0] < 1e-4 and errs["f32"][1] <= 1e-3
    assert errs["f16"][0] < 1e-2 and errs["f16"][1] <= 5e-2
