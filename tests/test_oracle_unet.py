"""Pins of the oracle's U-Net, its reverse mode and the physics-informed loss.

Layers are pinned to library routines (torch.nn.functional in FP64 on the CPU)
and to a brute-force loop; the network to exact properties (positive
homogeneity, translation equivariance, input scaling); the reverse mode to
central finite differences and to torch.autograd; the loss to its definition
as the backward error of the prediction (Section 3.3).
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import helmholtz as hz
from oracle import unet
from synth import C_REF, H_10PPW, he_uniform, rng_for, skull_ring_velocity, box_smoothed_noise

torch.set_num_threads(4)


def rand(*shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv3_matches_torch_and_loops():
    x, W, b = rand(2, 3, 7, 9, seed=1), rand(4, 3, 3, 3, seed=2), rand(4, seed=3)
    out = unet.conv3(x, W, b)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(W), torch.from_numpy(b), padding=1).numpy()
    assert np.max(np.abs(out - ref)) < 1e-13
    # brute force, one output entry at a time
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    for (bb, o, y, xx) in [(0, 0, 0, 0), (1, 3, 6, 8), (0, 2, 3, 4)]:
        s = b[o]
        for c in range(3):
            for dy in range(3):
                for dx in range(3):
                    s += W[o, c, dy, dx] * xp[bb, c, y + dy, xx + dx]
        assert abs(out[bb, o, y, xx] - s) < 1e-13


def test_conv1_convT2_pool_match_torch():
    x = rand(2, 6, 4, 5, seed=4)
    W1, b1 = rand(3, 6, 1, 1, seed=5), rand(3, seed=6)
    ref = F.conv2d(torch.from_numpy(x), torch.from_numpy(W1), torch.from_numpy(b1)).numpy()
    assert np.max(np.abs(unet.conv1(x, W1, b1) - ref)) < 1e-13
    WT, bT = rand(6, 5, 2, 2, seed=7), rand(5, seed=8)
    ref = F.conv_transpose2d(torch.from_numpy(x), torch.from_numpy(WT), torch.from_numpy(bT), stride=2).numpy()
    assert np.max(np.abs(unet.convT2(x, WT, bT) - ref)) < 1e-13
    x2 = rand(2, 3, 6, 8, seed=9)
    ref = F.avg_pool2d(torch.from_numpy(x2), 2).numpy()
    assert np.max(np.abs(unet.avgpool2(x2) - ref)) < 1e-15


def test_param_count_matches_architecture():
    # 4 levels, 32 base channels, 5 inputs: counted by hand layer by layer
    # enc: 1472 + 9248 + 18496 + 36928 + 73856 + 147584 + 295168 + 590080
    # dec2: 131200 + 295040 + 147584, dec1: 32832 + 73792 + 36928, dec0: 8224 + 18464 + 9248, head 66
    specs = unet.layer_specs(4, 32, 5)
    assert unet.param_count(specs) == 1_926_210
    # and torch's own modules of the same shapes agree
    n = 0
    for name, kind, ci, co in specs:
        if kind == "convT2":
            mod = torch.nn.ConvTranspose2d(ci, co, 2, stride=2)
        else:
            mod = torch.nn.Conv2d(ci, co, 3 if kind == "conv3" else 1)
        n += sum(p.numel() for p in mod.parameters())
    assert n == 1_926_210


def torch_unet(theta, specs, X):
    """Independent re-statement of the architecture with torch.nn.functional (FP64, CPU)."""
    P = {k: (torch.from_numpy(np.ascontiguousarray(w)), torch.from_numpy(np.ascontiguousarray(b)))
         for k, (w, b) in unet.unpack(theta, specs).items()}
    L = sum(1 for s in specs if s[0].startswith("enc")) // 2
    h = X
    skips = []
    for l in range(L):
        if l:
            h = F.avg_pool2d(h, 2)
        h = F.relu(F.conv2d(h, *P[f"enc{l}a"], padding=1))
        h = F.relu(F.conv2d(h, *P[f"enc{l}b"], padding=1))
        skips.append(h)
    for l in range(L - 2, -1, -1):
        u = F.conv_transpose2d(h, *P[f"up{l}"], stride=2)
        h = torch.cat([skips[l], u], 1)
        h = F.relu(F.conv2d(h, *P[f"dec{l}a"], padding=1))
        h = F.relu(F.conv2d(h, *P[f"dec{l}b"], padding=1))
    return F.conv2d(h, *P["head"])


def torch_unet_bf16_storage(theta, specs, X):
    """The same architecture with every stored activation cast FP64 -> FP32 -> bfloat16 -> FP64 by
    torch (input, 3x3 outputs after ReLU, transposed-conv outputs; pooling from the uncast value)."""
    q = lambda t: t.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    P = {k: (torch.from_numpy(np.ascontiguousarray(w)), torch.from_numpy(np.ascontiguousarray(b)))
         for k, (w, b) in unet.unpack(theta, specs).items()}
    L = sum(1 for s in specs if s[0].startswith("enc")) // 2
    h, raw = q(X), None
    skips = []
    for l in range(L):
        if l:
            h = q(F.avg_pool2d(raw, 2))
        h = q(F.relu(F.conv2d(h, *P[f"enc{l}a"], padding=1)))
        raw = F.relu(F.conv2d(h, *P[f"enc{l}b"], padding=1))
        skips.append(q(raw))
    h = skips[-1]
    for l in range(L - 2, -1, -1):
        u = q(F.conv_transpose2d(h, *P[f"up{l}"], stride=2))
        h = torch.cat([skips[l], u], 1)
        h = q(F.relu(F.conv2d(h, *P[f"dec{l}a"], padding=1)))
        h = q(F.relu(F.conv2d(h, *P[f"dec{l}b"], padding=1)))
    return F.conv2d(h, *P["head"])


def test_bf16_activation_rounding():
    # round to nearest even at 8 significant bits; torch's float32 -> bfloat16 cast agrees
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0, 1e-30, 3.0e38, np.inf, np.nan])
    r = unet.bf16_activation(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6 and r[3] == -2.5 and r[4] == 0.0
    assert np.isinf(r[7]) and np.isnan(r[8])
    y = np.random.default_rng(3).standard_normal(10000) * 10.0 ** np.random.default_rng(4).uniform(-5, 5, 10000)
    ref = torch.from_numpy(y).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16_activation(y), ref)


@pytest.mark.parametrize("levels,base,in_ch", [(2, 4, 2), (3, 4, 5)])
def test_forward_bf16_activation_storage_matches_torch(levels, base, in_ch):
    specs = unet.layer_specs(levels, base, in_ch)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(levels)).astype(np.float64)
    X = rand(2, in_ch, 16, 24, seed=levels)
    out = unet.forward(theta, specs, X, act_round=unet.bf16_activation)
    ref = torch_unet_bf16_storage(theta, specs, torch.from_numpy(X)).numpy()
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
    exact = unet.forward(theta, specs, X)
    assert np.array_equal(unet.forward(theta, specs, X, act_round=lambda a: a), exact)
    assert np.abs(out - exact).max() > 1e-4 * np.abs(exact).max()     # the rounding is applied


@pytest.mark.parametrize("levels,base,in_ch", [(2, 4, 2), (3, 4, 5), (4, 2, 5)])
def test_forward_matches_torch_composition(levels, base, in_ch):
    specs = unet.layer_specs(levels, base, in_ch)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(levels)).astype(np.float64)
    X = rand(2, in_ch, 16, 24, seed=levels)
    out = unet.forward(theta, specs, X)
    ref = torch_unet(theta, specs, torch.from_numpy(X)).numpy()
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


def test_forward_positive_homogeneity_without_bias():
    specs = unet.layer_specs(3, 4, 2)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(3)).astype(np.float64)
    P = unet.unpack(theta, specs)
    for _, (w, b) in P.items():
        b[:] = 0.0
    X = rand(1, 2, 16, 16, seed=4)
    a = 3.7
    assert np.allclose(unet.forward(theta, specs, a * X), a * unet.forward(theta, specs, X), rtol=1e-12, atol=1e-12)


def test_forward_translation_equivariance():
    # shifting the input by a multiple of 2^(L-1) shifts the output, away from the zero-padded border
    specs = unet.layer_specs(3, 4, 2)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(5)).astype(np.float64)
    # (the receptive field of 3 levels is under 48 pixels, so the centre of a 160 grid is unaffected)
    X = np.zeros((1, 2, 160, 160))
    X[0, :, 72:80, 72:80] = rand(2, 8, 8, seed=6)
    Xs = np.roll(X, (4, 8), axis=(2, 3))
    o, os_ = unet.forward(theta, specs, X), unet.forward(theta, specs, Xs)
    d = np.roll(o, (4, 8), axis=(2, 3)) - os_
    assert np.max(np.abs(d[:, :, 60:100, 60:100])) < 1e-12
    assert np.max(np.abs(o[:, :, 60:100, 60:100] - os_[:, :, 60:100, 60:100])) > 1e-3


def small_problem(seed, nx=24, p=4):
    nt = nx + 2 * p
    c = skull_ring_velocity(nt, p, rng_for(9, 0, seed), rings=1)
    return hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF)


def test_precond_scale_equivariance_and_zero():
    specs = unet.layer_specs(2, 4, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(7)).astype(np.float64)
    P = small_problem(0, nx=22, p=4)     # 30 x 30: padded to 30 (multiple of 2)
    v = box_smoothed_noise(P.nx, np.random.default_rng(8))
    z = unet.precond_apply(theta, specs, P, v)
    z2 = unet.precond_apply(theta, specs, P, 2.5 * v)
    assert np.allclose(z2, 2.5 * z, rtol=1e-12, atol=1e-14)
    assert np.all(unet.precond_apply(theta, specs, P, 0 * v) == 0)


def fd_check(specs, theta, problems, rs, squared, ndir=3, eps=1e-6, seed=0, ops=None):
    loss, _, g = unet.loss_and_grad(theta, specs, problems, rs, squared=squared, ops=ops)
    rng = np.random.default_rng(seed)
    errs = []
    for _ in range(ndir):
        d = rng.standard_normal(theta.size)
        d /= np.linalg.norm(d)
        lp = unet.loss_and_grad(theta + eps * d, specs, problems, rs, squared=squared, need_grad=False, ops=ops)[0]
        lm = unet.loss_and_grad(theta - eps * d, specs, problems, rs, squared=squared, need_grad=False, ops=ops)[0]
        fd = (lp - lm) / (2 * eps)
        an = float(g @ d)
        errs.append(abs(fd - an) / max(abs(an), 1e-12))
    return max(errs)


@pytest.mark.parametrize("squared", [False, True])
def test_gradient_finite_differences_32grid_8ch(squared):
    # 4 levels, 8 base channels, 5 inputs on a 32 x 32 grid (24 interior + 4 PML), FP64
    specs = unet.layer_specs(4, 8, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(11)).astype(np.float64)
    problems = [small_problem(s, nx=24, p=4) for s in range(2)]
    rs = np.stack([box_smoothed_noise(32, np.random.default_rng(20 + s)) for s in range(2)])
    assert fd_check(specs, theta, problems, rs, squared) < 1e-6


@pytest.mark.parametrize("squared", [False, True])
def test_gradient_finite_differences_spectral_operator(squared):
    # the loss on the Fourier-differentiation operator (Section 2.1): its gradient, through that
    # operator's adjoint, against central differences; and the operator really is the other one
    from oracle import spectral
    specs = unet.layer_specs(3, 8, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(12)).astype(np.float64)
    problems = [small_problem(s, nx=24, p=4) for s in range(2)]
    rs = np.stack([box_smoothed_noise(32, np.random.default_rng(30 + s)) for s in range(2)])
    assert fd_check(specs, theta, problems, rs, squared, ops=spectral) < 1e-6
    l_fd = unet.loss_and_grad(theta, specs, problems, rs, squared=squared, need_grad=False)[0]
    l_sp = unet.loss_and_grad(theta, specs, problems, rs, squared=squared, need_grad=False, ops=spectral)[0]
    assert abs(l_fd - l_sp) > 1e-3 * l_fd


def test_gradient_matches_torch_autograd():
    specs = unet.layer_specs(3, 4, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(12)).astype(np.float64)
    problems = [small_problem(s, nx=24, p=4) for s in range(2)]
    rs = np.stack([box_smoothed_noise(32, np.random.default_rng(30 + s)) for s in range(2)])
    loss, _, g = unet.loss_and_grad(theta, specs, problems, rs)
    # autograd over an independent torch statement of the same loss, with dense operators
    th = torch.tensor(theta, requires_grad=True)
    # rebuild parameters from the torch leaf in the same flat order
    P, off = {}, 0
    for name, kind, ci, co in specs:
        shp = unet.weight_shape(kind, ci, co)
        nw = int(np.prod(shp))
        P[name] = (th[off:off + nw].reshape(shp), th[off + nw:off + nw + co])
        off += nw + co
    L = 3
    total = 0
    for b, p in enumerate(problems):
        r = rs[b]
        s = np.linalg.norm(r) / np.sqrt(r.size)
        sx, sy = p.sigma_nodes()
        X = torch.tensor(np.stack([r.real / s, r.imag / s, p.c / p.c_ref, sx, sy])[None])
        h, skips = X, []
        for l in range(L):
            if l:
                h = F.avg_pool2d(h, 2)
            h = F.relu(F.conv2d(h, *P[f"enc{l}a"], padding=1))
            h = F.relu(F.conv2d(h, *P[f"enc{l}b"], padding=1))
            skips.append(h)
        for l in range(L - 2, -1, -1):
            u = F.conv_transpose2d(h, *P[f"up{l}"], stride=2)
            h = torch.cat([skips[l], u], 1)
            h = F.relu(F.conv2d(h, *P[f"dec{l}a"], padding=1))
            h = F.relu(F.conv2d(h, *P[f"dec{l}b"], padding=1))
        out = F.conv2d(h, *P["head"])[0]
        z = s * torch.complex(out[0], out[1]).reshape(-1)
        A = torch.tensor(hz.assemble_dense(p))
        q = A @ z - torch.tensor(r.ravel())
        total = total + torch.linalg.vector_norm(q) / np.linalg.norm(r)
    total = total / len(problems)
    total.backward()
    assert abs(total.item() - loss) < 1e-12 * loss
    assert np.max(np.abs(th.grad.numpy() - g)) <= 1e-11 * np.max(np.abs(g))


def test_loss_is_backward_error_of_prediction():
    # Section 3.3: the (squared) loss equals eta_b of the prediction u = N(b) for A u = b
    specs = unet.layer_specs(2, 4, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(13)).astype(np.float64)
    p = small_problem(3, nx=22, p=4)
    b = box_smoothed_noise(30, np.random.default_rng(14))
    u = unet.precond_apply(theta, specs, p, b)
    A = hz.assemble_dense(p)
    eta = np.linalg.norm(A @ u.ravel() - b.ravel()) / np.linalg.norm(b)
    loss, _, _ = unet.loss_and_grad(theta, specs, [p], b[None], need_grad=False)
    loss2, _, _ = unet.loss_and_grad(theta, specs, [p], b[None], squared=True, need_grad=False)
    assert loss == pytest.approx(eta, rel=1e-12)
    assert loss2 == pytest.approx(eta ** 2, rel=1e-12)
