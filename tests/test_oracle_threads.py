"""The oracle's optional OpenMP pixel and probe loops: every iteration reads
shared inputs and writes only its own outputs, so a whole chain (probe
update, G-buffer, initial, temporal, two spatial passes, shading, path
tracer) gives bitwise the same results on 1 thread and on several."""
import dataclasses

import numpy as np
import pytest

import oracle as o
from paper_2108_05263_amd import scenegen as sg


def _chain(threads):
    assert o.set_threads(threads) == threads
    try:
        cfg = sg.CONFIGS["tiny"]
        sc = sg.make_scene(cfg)
        grid = sg.make_probe_grid(cfg)
        irr, dep = o.fill_probes(sc, grid, sg.ProbeUpdate(rays=48, fill_passes=2, fill_rays=48), seed=3)
        pr = dataclasses.replace(cfg.params, temporal=True, n_spatial=2, M_light=2)
        seq = o.Sequence(sc, grid, irr, dep, pr, 7)
        out = [irr, dep]
        for f in range(2):
            img, st = seq.frame(sg.make_camera(cfg, f, 48, 40), f)
            out += [img] + [st[k] for k in sorted(st) if isinstance(st[k], np.ndarray)]
        gb = st["gbuffer"]
        out.append(o.path_trace(sc, gb, np.arange(0, 48 * 40, 7), 3, 5))
        return out
    finally:
        o.set_threads(1)


@pytest.mark.skipif(not o.lib().o_openmp(), reason="oracle built without OpenMP")
def test_threads_bitwise_identical():
    one, many = _chain(1), _chain(6)
    assert len(one) == len(many) > 8
    for a, b in zip(one, many):
        assert a.shape == b.shape
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
