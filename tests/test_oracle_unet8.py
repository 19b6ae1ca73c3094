"""Pins of the oracle's second network (the paper's 8x8 stride-2 layer set, Table 2): each layer
against torch.nn.functional, the parameter count against torch's own modules, the whole forward
against an independent torch composition, positive homogeneity, translation equivariance by the
network's stride and the preconditioner's scale equivariance."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import helmholtz as hz
from oracle import unet8
from synth import C_REF, H_10PPW, box_smoothed_noise, rng_for, skull_ring_velocity


def rand(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def test_layers_match_torch():
    x = rand(2, 5, 24, 40, seed=1)
    W = rand(7, 5, 8, 8, seed=2)
    b = rand(7, seed=3)
    y = unet8.down(x, W, b)
    assert y.shape == (2, 7, 12, 20)
    yt = F.conv2d(torch.tensor(x), torch.tensor(W), torch.tensor(b), stride=2, padding=3).numpy()
    assert np.max(np.abs(y - yt)) <= 1e-12 * np.max(np.abs(yt))
    Wt = rand(5, 6, 8, 8, seed=4)
    bt = rand(6, seed=5)
    u = unet8.up(x, Wt, bt)
    assert u.shape == (2, 6, 48, 80)
    ut = F.conv_transpose2d(torch.tensor(x), torch.tensor(Wt), torch.tensor(bt), stride=2, padding=3).numpy()
    assert np.max(np.abs(u - ut)) <= 1e-12 * np.max(np.abs(ut))
    a = 0.3
    assert np.array_equal(unet8.prelu(x, a), F.prelu(torch.tensor(x), torch.tensor([a], dtype=torch.float64)).numpy())
    W1 = rand(2, 5, 1, 1, seed=6)
    c1 = F.conv2d(torch.tensor(x), torch.tensor(W1), torch.tensor(b[:2])).numpy()
    assert np.max(np.abs(unet8.conv1(x, W1, b[:2]) - c1)) <= 1e-13 * np.max(np.abs(c1))


def test_param_count_matches_torch_modules():
    specs = unet8.layer_specs()
    n = 0
    for _, kind, ci, co in specs:
        if kind == "down":
            mods = [torch.nn.Conv2d(ci, co, 8, stride=2, padding=3), torch.nn.PReLU()]
        elif kind == "up":
            mods = [torch.nn.ConvTranspose2d(ci, co, 8, stride=2, padding=3), torch.nn.PReLU()]
        else:
            mods = [torch.nn.Conv2d(ci, co, 1)]
        n += sum(p.numel() for m in mods for p in m.parameters())
    assert n == unet8.param_count(specs) == 665_930


def torch_unet8(theta, specs, X):
    """Independent statement of the same graph with torch modules' functional forms (FP64)."""
    P, off = {}, 0
    t = torch.from_numpy(np.asarray(theta, np.float64))
    for name, kind, ci, co in specs:
        shp = unet8.weight_shape(kind, ci, co)
        nw = int(np.prod(shp))
        W = t[off:off + nw].reshape(shp)
        b = t[off + nw:off + nw + co]
        a = t[off + nw + co:off + nw + co + 1] if kind != "conv1" else None
        P[name] = (W, b, a)
        off += nw + co + (kind != "conv1")
    depth = 4
    h = torch.from_numpy(X)
    skips = [h]
    for l in range(1, depth + 1):
        W, b, a = P[f"down{l}"]
        h = F.prelu(F.conv2d(h, W, b, stride=2, padding=3), a)
        skips.append(h)
    W, b, a = P[f"up{depth - 1}"]
    h = F.prelu(F.conv_transpose2d(h, W, b, stride=2, padding=3), a)
    for l in range(depth - 2, -1, -1):
        W, b, a = P[f"up{l}"]
        h = F.prelu(F.conv_transpose2d(torch.cat([skips[l + 1], h], 1), W, b, stride=2, padding=3), a)
    W, b, _ = P["head"]
    return F.conv2d(h, W, b).numpy()


def test_forward_matches_torch_composition():
    specs = unet8.layer_specs()
    theta = unet8.init_theta(specs, np.random.default_rng(7)).astype(np.float64)
    off = 0
    for i, (_, kind, ci, co) in enumerate(specs):    # a different slope in every layer
        off += unet8.layer_len(kind, ci, co)
        if kind != "conv1":
            theta[off - 1] = 0.05 * (i + 1)
    P = unet8.unpack(theta, specs)
    assert [P[n][2] for n, k, _, _ in specs if k != "conv1"] == [0.05 * (i + 1) for i in range(8)]
    X = rand(2, 5, 48, 32, seed=8)
    o = unet8.forward(theta, specs, X)
    ot = torch_unet8(theta, specs, X)
    assert o.shape == (2, 2, 48, 32)
    assert np.max(np.abs(o - ot)) <= 1e-12 * np.max(np.abs(ot))
    assert len(P) == 9


def test_positive_homogeneity_without_bias():
    specs = unet8.layer_specs()
    theta = unet8.init_theta(specs, np.random.default_rng(9)).astype(np.float64)
    off = 0
    for _, kind, ci, co in specs:           # zero every bias
        nw = int(np.prod(unet8.weight_shape(kind, ci, co)))
        theta[off + nw:off + nw + co] = 0.0
        off += unet8.layer_len(kind, ci, co)
    X = rand(1, 5, 32, 32, seed=10)
    o = unet8.forward(theta, specs, X)
    assert np.allclose(unet8.forward(theta, specs, 3.5 * X), 3.5 * o, rtol=1e-12, atol=1e-13 * np.abs(o).max())


def test_translation_equivariance_by_the_stride():
    specs = unet8.layer_specs()
    theta = unet8.init_theta(specs, np.random.default_rng(11)).astype(np.float64)
    X = rand(1, 5, 288, 288, seed=12)
    o = unet8.forward(theta, specs, X)
    os_ = unet8.forward(theta, specs, np.roll(X, (16, 32), axis=(2, 3)))
    d = np.roll(o, (16, 32), axis=(2, 3)) - os_
    # away from the zero padding (the receptive field spans about 120 nodes each way)
    assert np.max(np.abs(d[:, :, 136:152, 136:152])) <= 1e-12 * np.abs(o).max()
    assert np.max(np.abs(o[:, :, 136:152, 136:152] - os_[:, :, 136:152, 136:152])) > 1e-3


def test_precond_scale_equivariance_zero_and_padding():
    specs = unet8.layer_specs()
    theta = unet8.init_theta(specs, np.random.default_rng(13)).astype(np.float64)
    nt, p = 30, 4                            # 30 x 30: padded to 32 (a multiple of 16)
    c = skull_ring_velocity(nt, p, rng_for(9, 0, 0), rings=1)
    P = hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF)
    v = box_smoothed_noise(nt, np.random.default_rng(14))
    z = unet8.precond_apply(theta, specs, P, v)
    assert z.shape == (30, 30)
    assert np.allclose(unet8.precond_apply(theta, specs, P, 2.5 * v), 2.5 * z, rtol=1e-12, atol=1e-14)
    assert np.all(unet8.precond_apply(theta, specs, P, 0 * v) == 0)


def test_backward_matches_torch_autograd():
    # the reverse mode of the whole network against autograd over the independent torch statement,
    # with a different PReLU slope of either sign in every layer
    specs = unet8.layer_specs(3, 32, 5)
    theta = unet8.init_theta(specs, np.random.default_rng(21)).astype(np.float64)
    r = np.random.default_rng(22)
    off = 0
    for _, kind, ci, co in specs:
        off += unet8.layer_len(kind, ci, co)
        if kind != "conv1":
            theta[off - 1] = r.uniform(-0.3, 0.6)
    X = rand(2, 5, 32, 48, seed=23)
    gout = rand(2, 2, 32, 48, seed=24)
    out, cache = unet8.forward(theta, specs, X, keep=True)
    g = unet8.backward(theta, specs, cache, gout)
    th = torch.tensor(theta, requires_grad=True)

    def torch_net(t):
        P, o = {}, 0
        for name, kind, ci, co in specs:
            shp = unet8.weight_shape(kind, ci, co)
            nw = int(np.prod(shp))
            P[name] = (t[o:o + nw].reshape(shp), t[o + nw:o + nw + co],
                       t[o + nw + co:o + nw + co + 1] if kind != "conv1" else None)
            o += unet8.layer_len(kind, ci, co)
        h = torch.from_numpy(X)
        skips = [h]
        for l in range(1, 4):
            W, b, a = P[f"down{l}"]
            h = F.prelu(F.conv2d(h, W, b, stride=2, padding=3), a)
            skips.append(h)
        W, b, a = P["up2"]
        h = F.prelu(F.conv_transpose2d(h, W, b, stride=2, padding=3), a)
        for l in (1, 0):
            W, b, a = P[f"up{l}"]
            h = F.prelu(F.conv_transpose2d(torch.cat([skips[l + 1], h], 1), W, b, stride=2, padding=3), a)
        W, b, _ = P["head"]
        return F.conv2d(h, W, b)

    y = torch_net(th)
    assert np.max(np.abs(y.detach().numpy() - out)) <= 1e-12 * np.abs(out).max()
    (y * torch.from_numpy(gout)).sum().backward()
    assert np.max(np.abs(th.grad.numpy() - g)) <= 1e-11 * np.max(np.abs(g))


@pytest.mark.parametrize("squared", [False, True])
def test_loss_gradient_finite_differences(squared):
    # the physics-informed loss through A and this network: central differences along three random
    # directions (FP64, 32 x 32 grid: 24 interior + 4 PML, depth 3)
    specs = unet8.layer_specs(3, 32, 5)
    theta = unet8.init_theta(specs, np.random.default_rng(25)).astype(np.float64)
    probs, rs = [], []
    for s in range(2):
        c = skull_ring_velocity(32, 4, rng_for(9, 0, 40 + s), rings=1)
        probs.append(hz.Problem(c, 4, H_10PPW, 1.0, 2.0, C_REF))
        rs.append(box_smoothed_noise(32, np.random.default_rng(50 + s)))
    rs = np.stack(rs)
    loss, per, g = unet8.loss_and_grad(theta, specs, probs, rs, squared=squared)
    assert np.isclose(loss, per.mean())
    rng = np.random.default_rng(26)
    for _ in range(3):
        d = rng.standard_normal(theta.size)
        d /= np.linalg.norm(d)
        eps = 1e-6
        lp = unet8.loss_and_grad(theta + eps * d, specs, probs, rs, squared=squared, need_grad=False)[0]
        lm = unet8.loss_and_grad(theta - eps * d, specs, probs, rs, squared=squared, need_grad=False)[0]
        fd = (lp - lm) / (2 * eps)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
