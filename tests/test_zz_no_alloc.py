"""The allocation-free training step (gi_mlp_train_step_noalloc) against the
training step with a caller workspace (gi_mlp_train_step): same kernels, so
every output is bit-identical.  Two calls in a row, the second with a
smaller batch (the scratch keeps the first call's contents, which the
second must not read), then the size limit."""
import sys

import numpy as np
import pytest
import torch

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu

LO, HI = np.zeros(3, np.float32), np.array([8.0, 8.0, 8.0], np.float32)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gi():
    from paper_2108_05263_amd import gi as m
    m.load()
    assert torch.cuda.is_available()
    return m


def _batch(gi, n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 8.0, (n, 3)).astype(np.float32)
    nrm = rng.normal(size=(n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    tgt = rng.uniform(0.0, 2.0, (n, 3)).astype(np.float32)
    valid = rng.random(n) < 0.85
    tgt[~valid] = 0.0
    q = rng.uniform(0.0, 1.5, (n, 3)).astype(np.float32)
    z = np.zeros((n, 1), np.float32)
    b = gi.MlpBatch(n)
    b.pos.copy_(torch.from_numpy(np.concatenate([pos, z], 1)))
    b.nrm.copy_(torch.from_numpy(np.concatenate([nrm, z], 1)))
    b.target.copy_(torch.from_numpy(np.concatenate([tgt, valid[:, None].astype(np.float32)], 1)))
    b.qprobe.copy_(torch.from_numpy(np.concatenate([q, z], 1)))
    return b


def _state(m):
    torch.cuda.synchronize()
    out = {k: getattr(m, k).cpu().numpy().copy() for k in ("params", "adam_m", "adam_v", "ema", "scales", "state")}
    out["weights"] = m.weights.cpu().numpy().copy()
    return out


def _same(a, b, label):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{label}: {k} differs"


def test_noalloc_train_step_matches_workspace_step(gi):
    params = M.init_params_philox(5).astype(np.float32)
    mk = []
    for _ in range(2):
        m = gi.Mlp(LO, HI, precision="bf16", mode="auto", warmup_steps=1, ema_decay=0.99)
        m.load_params(params)
        mk.append(m)
    ref, dut = mk
    for t, n, seed in ((1, 16384, 11), (2, 3000, 12)):
        log(f"noalloc train step t={t} n={n}")
        b = _batch(gi, n, seed)
        ws = gi.train_workspace(n)
        gi.mlp_train_step(ref, b, t, 1e-2, ws)
        gi.mlp_train_step_noalloc(dut, b, t, 1e-2)
        sr, sd = _state(ref), _state(dut)
        _same(sr, sd, f"step {t} (n={n})")
        assert sd["state"][1] == t                                   # Adam steps taken
        assert not np.array_equal(sd["params"], params)              # the step moved the parameters
        del ws


def test_noalloc_train_step_rejects_oversized_batch(gi):
    m = gi.Mlp(LO, HI, precision="bf16")
    m.init(3)
    n = 16384 + 1
    b = gi.MlpBatch(n)
    with pytest.raises(gi.GiError):
        gi.mlp_train_step_noalloc(m, b, 1, 1e-2)
    torch.cuda.synchronize()
    assert m.state_words()["steps"] == 0
