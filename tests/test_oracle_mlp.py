"""Pins of the learned-cache oracle (oracle/mlp_ref.py) against independent
implementations:

* BF16 / FP8-E4M3FN rounding == torch's casts;
* encoding identities (sin^2 + cos^2 = 1, frequency doubling, raw value);
* FP64 forward == torch Linear/ReLU stack; backward == torch autograd of the
  relative-L2 loss with a stop-gradient denominator; central finite
  differences agree with the backward;
* BF16 forward/backward == torch autograd where every GEMM operand (and
  back-propagated gradient) passes through a BF16 rounding function;
* FP8 forward == torch float8_e4m3fn casts with per-layer scales;
* Adam == torch.optim.Adam (float64);
* training labels in a closed form: in a room whose walls emit L and whose
  probes are empty, every label equals L exactly.
"""
import math

import numpy as np
import pytest
import torch

import oracle as o
from oracle import mlp_ref as M
from paper_2108_05263_amd import scenegen as sg



@pytest.fixture(autouse=True)
def _float64_default():
    """torch's default dtype is float64 inside this module's tests only (its
    reference layers are built in FP64); other modules keep float32."""
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def _batch(n=64, seed=0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 8.0, (n, 3))
    nrm = rng.normal(size=(n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return M.encode(pos, nrm, np.zeros(3), np.full(3, 8.0))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.normal(0, 1e-3, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -1e-30]])
    # exact ties: values halfway between two bf16 numbers
    b = rng.integers(0x3C00, 0x4300, 200).astype(np.uint32)       # bf16 patterns in [2^-7, 2^7)
    ties = ((b << 16) | 0x8000).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(x), ref)


def test_fp8_rounding_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 50, 5000), rng.normal(0, 0.01, 2000),
                        np.arange(-64, 64) / 32.0 + 1.0 / 64.0,      # ties at various exponents
                        [0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11]])
    x = np.clip(x, -448, 448)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(M.round_fp8_e4m3(x), ref)
    assert np.all(np.abs(M.round_fp8_e4m3([1000.0, -900.0])) == 448.0)


def test_encoding_identities():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 8, (50, 3))
    nrm = rng.normal(size=(50, 3))
    lo, hi = np.zeros(3), np.full(3, 8.0)
    X = M.encode(pos, nrm, lo, hi)
    assert X.shape == (50, 78) and M.N_ENC == 78
    v = np.concatenate([pos / 8.0, nrm], axis=1)
    for i in range(6):
        assert np.allclose(X[:, 13 * i], v[:, i], rtol=0, atol=1e-15)
        for j in range(6):
            s, c = X[:, 13 * i + 1 + 2 * j], X[:, 13 * i + 2 + 2 * j]
            assert np.allclose(s * s + c * c, 1.0, atol=1e-12)
            if j > 0:
                sp, cp = X[:, 13 * i + 2 * j - 1], X[:, 13 * i + 2 * j]
                assert np.allclose(s, 2 * sp * cp, atol=1e-12)
        # j = 0 is sin(pi v): zero at v = 0 and v = 1
    z = M.encode(np.zeros((1, 3)), np.zeros((1, 3)), lo, hi)
    assert np.allclose(z[0, 1::13][:6], 0.0) and np.allclose(z[0, 2::13][:6], 1.0)


def _torch_net(params):
    layers = []
    for (W, b), (i, n) in zip(M.split(params), M.LAYERS):
        lin = torch.nn.Linear(i, n)
        lin.weight.data = torch.tensor(W)
        lin.bias.data = torch.tensor(b)
        layers.append(lin)
    return layers


def _torch_forward(layers, X, rnd=None):
    h = X
    for li, lin in enumerate(layers):
        if rnd is not None:
            h = rnd(h) @ rnd(lin.weight).T + lin.bias
        else:
            h = lin(h)
        if li < len(layers) - 1:
            h = torch.relu(h)
    return h


def _torch_loss(out, target, valid):
    w = torch.tensor(valid, dtype=torch.float64)[:, None]
    den = out.detach() ** 2 + 0.01
    return (((out - target) ** 2 / den) * w).sum() / (max(valid.sum(), 1) * 3)


def test_fp64_forward_backward_match_torch_and_fd():
    params = M.init_params(7)
    assert params.size == M.N_PARAMS == 17731
    X = _batch(48)
    rng = np.random.default_rng(4)
    target = rng.uniform(0, 2, (48, 3))
    valid = rng.random(48) > 0.2
    out, cache = M.forward(params, X)
    layers = _torch_net(params)
    tout = _torch_forward(layers, torch.tensor(X))
    assert np.allclose(out, tout.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss, g = M.loss_and_grad_out(out, target, valid)
    tl = _torch_loss(tout, torch.tensor(target), valid)
    assert loss == pytest.approx(float(tl), rel=1e-12)
    grad = M.backward(params, cache, g)
    tl.backward()
    tg = np.concatenate([np.concatenate([l.weight.grad.numpy().ravel(), l.bias.grad.numpy()]) for l in layers])
    assert np.allclose(grad, tg, rtol=1e-10, atol=1e-14)
    # central finite differences of the loss with the denominator frozen
    den_fixed = out * out + 0.01

    def loss_frozen(p):
        o_, _ = M.forward(p, X)
        w = valid.astype(np.float64)[:, None]
        return float((((o_ - target) ** 2 / den_fixed) * w).sum() / (valid.sum() * 3))
    for idx in rng.choice(M.N_PARAMS, 25, replace=False):
        h = 1e-6
        pp, pm = params.copy(), params.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (loss_frozen(pp) - loss_frozen(pm)) / (2 * h)
        assert fd == pytest.approx(grad[idx], rel=1e-5, abs=1e-10)


class _RoundFwd(torch.autograd.Function):
    """BF16 rounding of a GEMM operand (forward only)."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGradIn(torch.autograd.Function):
    """Identity forward; BF16 rounding of the gradient that enters the GEMM
    backward products (dW = g^T x and dx = g W take g in BF16)."""

    @staticmethod
    def forward(ctx, x):
        return x

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_bf16_training_semantics_match_torch():
    params = M.init_params(8)
    X = _batch(40, 5)
    rng = np.random.default_rng(6)
    target = rng.uniform(0, 2, (40, 3))
    valid = np.ones(40, bool)
    out, cache = M.forward(params, X, prec="bf16")
    loss, g = M.loss_and_grad_out(out, target, valid)
    grad = M.backward(params, cache, g, prec="bf16")
    layers = _torch_net(params)
    h = torch.tensor(X)
    for li, lin in enumerate(layers):
        z = _RoundGradIn.apply(_RoundFwd.apply(h) @ _RoundFwd.apply(lin.weight).T) + lin.bias
        h = torch.relu(z) if li < len(layers) - 1 else z
    assert np.allclose(out, h.detach().numpy(), rtol=1e-12, atol=1e-12)
    tl = _torch_loss(h, torch.tensor(target), valid)
    tl.backward()
    tg = np.concatenate([np.concatenate([l.weight.grad.numpy().ravel(), l.bias.grad.numpy()]) for l in layers])
    assert np.allclose(grad, tg, rtol=1e-9, atol=1e-13)
    # BF16 output stays close to FP64
    ref, _ = M.forward(params, X)
    assert np.max(np.abs(out - ref)) < 0.05 * (np.max(np.abs(ref)) + 1e-3)


def test_fp8_scales_are_powers_of_two_covering_the_range():
    rng = np.random.default_rng(12)
    for amax in list(rng.uniform(1e-6, 1e4, 200)) + [448.0, 224.0, 448.0 * 2 ** -20, 3.0 * 2 ** -130]:
        s = M.fp8_scale(amax)
        m, e = math.frexp(s)
        assert m == 0.5                                  # a power of two
        assert amax <= 448.0 * s and amax > 224.0 * s    # the smallest that covers amax
    assert M.fp8_scale(0.0) == 1.0 and M.fp8_scale(float("inf")) == 1.0
    for x in list(rng.uniform(1e-8, 1e3, 200)) + [1.0, 0.5, 2.0 ** -40]:
        p = M.pow2_at_least(x)
        assert math.frexp(p)[0] == 0.5 and x <= p < 2 * x


def test_fp8_forward_matches_torch_casts():
    params = M.init_params(9)
    X = _batch(40, 7)
    amax = M.act_amax(params, X)
    sa = [a / 448.0 for a in amax]
    out, _ = M.forward(params, X, prec="fp8", act_scales=sa)
    h = torch.tensor(X)
    f8 = torch.float8_e4m3fn
    for li, (W, b) in enumerate(M.split(params)):
        # power-of-two scales: weights from amax|W|, activations rounded up
        sw = 2.0 ** math.ceil(math.log2(float(np.max(np.abs(W))) / 448.0))
        sa_l = 2.0 ** math.ceil(math.log2(sa[li]))
        a8 = (h / sa_l).clamp(-448, 448).to(torch.float32).to(f8).to(torch.float64)
        w8 = (torch.tensor(W) / sw).to(torch.float32).to(f8).to(torch.float64)
        h = (a8 @ w8.T) * (sw * sa_l) + torch.tensor(b)
        if li < 4:
            h = torch.relu(h)
    assert np.allclose(out, h.numpy(), rtol=1e-12, atol=1e-12)
    ref, _ = M.forward(params, X)
    assert np.max(np.abs(out - ref)) < 0.2 * (np.max(np.abs(ref)) + 1e-3)


def test_adam_matches_torch():
    rng = np.random.default_rng(10)
    p = rng.normal(size=300)
    m, v = np.zeros(300), np.zeros(300)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.99), eps=1e-8)
    for t in range(1, 8):
        g = rng.normal(size=300) * (0.1 * t)
        p, m, v = M.adam_step(p, m, v, g, t)
        tp.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_batch_labels_closed_form():
    # walls emit L and have albedo 0.5; every probe texel holds irradiance/pi
    # c: a label is the radiance arriving from another wall point, L_e + rho c
    # = L + c/2 exactly, and the probe value at the sample is c
    L = np.array([0.7, 1.1, 1.9], np.float32)
    c = np.array([0.25, 0.5, 1.5], np.float32)
    sc = sg.Scene(prims=np.zeros((0, 16), np.float32), has_room=True, room_lo=np.zeros(3, np.float32),
                  room_hi=np.full(3, 8.0, np.float32), wall_albedo=np.full(3, 0.5, np.float32),
                  sky=np.zeros(3, np.float32), eps=8e-4, wall_emit=L)
    cfg = sg.CONFIGS["tiny"]
    cam = sg.make_camera(cfg, 0, 24, 24)
    grid = sg.probe_grid((2, 2, 2), (0, 0, 0), 4.0)
    irr, dep = sg.empty_probe_textures(grid)
    irr[..., :3] = c
    dep[..., 0], dep[..., 1] = 1.0, 1.0
    gb = o.gbuffer(sc, cam)
    pos, nrm, tgt, valid, qp = o.mlp_batch(sc, 24, 24, gb, grid, irr, dep, 4, 300, 5, 0)
    assert valid.mean() > 0.9
    want = L.astype(np.float64) + 0.5 * c.astype(np.float64)
    assert np.allclose(tgt[valid], want, rtol=1e-14, atol=0)
    assert np.allclose(qp[valid], c.astype(np.float64), rtol=1e-14, atol=0)
    assert np.all(tgt[~valid] == 0) and np.all(qp[~valid] == 0)
    # inputs are candidates of the initial pass, on the walls, with unit normals
    on_wall = np.min(np.minimum(pos[valid], 8.0 - pos[valid]), axis=1)
    assert np.all(on_wall < 1e-6)
    assert np.allclose(np.linalg.norm(nrm[valid], axis=1), 1.0)


def test_c_forward_matches_numpy_oracle():
    """The C oracle's MLP (used as the resampling target) == the numpy oracle."""
    params = M.init_params(11)
    rng = np.random.default_rng(12)
    pos = rng.uniform(0, 8, (30, 3))
    nrm = rng.normal(size=(30, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    lo, hi = np.zeros(3, np.float32), np.full(3, 8.0, np.float32)
    X = M.encode(pos, nrm, lo, hi)
    for prec in ("f64", "bf16"):
        ref, _ = M.forward(params, X, prec=prec)
        got = o.mlp_forward(params, prec, lo, hi, pos, nrm)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12), prec


def test_constant_mlp_target_equals_constant_probes():
    """A network with zero weights outputs its last bias c everywhere; as a
    target it must give the same reservoirs and image as probes whose
    irradiance texels all hold c (the probe query's normalised blend of a
    constant is that constant)."""
    cfg = sg.CONFIGS["tiny"]
    sc = sg.make_scene(cfg)
    W, H = 32, 24
    cam = sg.make_camera(cfg, 0, W, H)
    grid = sg.make_probe_grid(cfg)
    c = np.array([0.25, 0.5625, 0.8125])            # exact in the binary16 texels
    params = np.zeros(M.N_PARAMS)
    params[-3:] = c
    lo, hi = sc.bounds()
    mlp = o.MlpTarget(params, lo, hi, prec="f64")
    irr, dep = sg.empty_probe_textures(grid)
    irr[..., :3] = c.astype(np.float32)
    dep[..., 0], dep[..., 1] = 1.0, 1.0
    gb = o.gbuffer(sc, cam)
    pr = sg.Params(M=8)
    r_mlp, d_mlp = o.resample_initial(sc, W, H, gb, grid, irr * 0, dep, pr, 3, 0, mlp=mlp)
    r_prb, d_prb = o.resample_initial(sc, W, H, gb, grid, irr, dep, pr, 3, 0)
    assert np.allclose(r_mlp, r_prb, rtol=1e-9, atol=1e-12)
    assert np.allclose(d_mlp, d_prb, rtol=1e-9, atol=1e-12)
    i_mlp = o.shade(sc, W, H, gb, grid, irr * 0, dep, r_mlp, d_mlp, pr, mlp=mlp)
    i_prb = o.shade(sc, W, H, gb, grid, irr, dep, r_prb, d_prb, pr)
    assert np.allclose(i_mlp, i_prb, rtol=1e-9, atol=1e-12)
    assert np.abs(i_mlp).max() > 0.1


def test_philox_init_distribution():
    """He-uniform initialisation: every weight in [-b, b) with b = sqrt(6/fan_in),
    zero biases, per-layer mean ~ 0 and variance ~ b^2/3 (uniform law)."""
    p = M.init_params_philox(5)
    for (W, b), (i, n) in zip(M.split(p), M.LAYERS):
        bound = math.sqrt(6.0 / i)
        assert np.all(b == 0)
        assert np.all(np.abs(W) <= bound * (1 + 1e-6))
        k = W.size
        assert abs(W.mean()) < 5 * bound / math.sqrt(3 * k)
        assert W.var() == pytest.approx(bound ** 2 / 3, rel=8 * math.sqrt(0.8 / k) + 0.01)
    # two seeds differ, one seed repeats
    assert not np.array_equal(p, M.init_params_philox(6))
    assert np.array_equal(p, M.init_params_philox(5))


def test_batch_inputs_are_initial_candidates():
    """A training input is candidate i = floor(u1 M) of pixel p = floor(u0 W H)
    of the initial pass: with M = 1 the initial reservoir holds exactly that
    candidate, so the sample's position equals the reservoir's y."""
    cfg = sg.CONFIGS["tiny"]
    sc = sg.make_scene(cfg)
    grid = sg.make_probe_grid(cfg)
    irr, dep = sg.empty_probe_textures(grid)
    irr[..., :3] = 0.5      # every candidate on a lit surface gets a positive weight
    dep[..., 0], dep[..., 1] = 1.0, 1.0
    W, H = 20, 16
    gb = o.gbuffer(sc, sg.make_camera(cfg, 0, W, H))
    res, _ = o.resample_initial(sc, W, H, gb, grid, irr, dep, sg.Params(M=1), 3, 2)
    pos, nrm, tgt, valid, qp = o.mlp_batch(sc, W, H, gb, grid, irr, dep, 1, 400, 3, 2)
    assert valid.mean() > 0.5
    for j in np.nonzero(valid)[0]:
        u = o.philox(3, [j, 2, 10, 0])
        p = int(((int(u[0]) >> 8) * W * H) >> 24)
        assert np.allclose(pos[j], res[p, 0:3], rtol=0, atol=1e-12)
        assert np.allclose(nrm[j], res[p, 3:6], rtol=0, atol=1e-12)
