"""GPU parity of the training step (no_loss_backward, no_adam_step) against the oracle's loss,
reverse mode and Adam."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from oracle import adam as oadam
from oracle import helmholtz as ohz
from oracle import unet
from synth import box_smoothed_noise, c3_batch, he_uniform, rng_for, skull_ring_velocity

from gpu_util import make_pair, rel, to_dev, to_np
from test_gpu_net import bf16_round


def batch(nx, p, B, seed=0):
    nt = nx + 2 * p
    ops, gps, rs = [], [], []
    for b in range(B):
        c = skull_ring_velocity(nt, p, rng_for(14, 0, 10 * seed + b), rings=1 + b % 3)
        op, gp = make_pair(c, p)
        ops.append(op)
        gps.append(gp)
        rs.append(box_smoothed_noise(nt, rng_for(14, 3, 10 * seed + b)))
    return ops, gps, np.stack(rs)


def run(levels, base, nx, p, B, prec, squared=False, seed=0):
    from paper_2607_16906_amd import hz
    ops, gps, rs = batch(nx, p, B, seed)
    specs = unet.layer_specs(levels, base, 5)
    theta = he_uniform(unet.init_shapes(specs), rng_for(14, 2, seed))
    net = hz.Net(levels, base, 5, theta)
    r = to_dev(rs.astype(np.complex64), torch.complex64)
    loss, per, grad = hz.loss_backward(net, gps, r, squared=squared, prec=prec)
    th = bf16_round(theta) if prec == "bf16" else theta.astype(np.float64)
    # the oracle sees the same FP32-rounded residuals as the GPU
    rr = rs.astype(np.complex64).astype(np.complex128)
    ref_loss, ref_per, ref_grad = unet.loss_and_grad(th, specs, ops, rr, squared=squared)
    return to_np(loss)[0], to_np(per), to_np(grad), ref_loss, ref_per, ref_grad, specs


@pytest.mark.parametrize("squared", [False, True])
def test_fp32_gradient_matches_oracle_small(squared):
    # the finite-difference configuration: 32 x 32 grid (24 + 4 PML), 8 base channels, 4 levels
    loss, per, g, rl, rp, rg, specs = run(4, 8, 24, 4, 2, "fp32", squared)
    assert abs(loss - rl) <= 1e-5 * rl
    assert np.max(np.abs(per - rp) / rp) <= 1e-5
    err = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"fp32 grad rel err {err:.2e}")
    assert err <= 1e-4
    # every layer, weights and bias, individually
    off = 0
    for name, kind, ci, co in specs:
        nw = int(np.prod(unet.weight_shape(kind, ci, co)))
        for a, b in ((off, off + nw), (off + nw, off + nw + co)):
            e = np.linalg.norm(g[a:b] - rg[a:b]) / max(np.linalg.norm(rg[a:b]), 1e-30)
            assert e <= 1e-3, (name, a, e)
        off += nw + co


def test_fp32_gradient_matches_oracle_ragged_32ch():
    # 3 levels, 32 channels, a grid whose padded size (44) leaves ragged tiles
    # (a pre-activation within FP32 rounding of zero can take the other side of its ReLU kink than
    # in FP64, so a few entries differ at O(1) of their own size: the bound is normwise)
    loss, per, g, rl, rp, rg, _ = run(3, 32, 30, 6, 3, "fp32", seed=1)
    assert abs(loss - rl) <= 1e-5 * rl
    err = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"fp32 grad rel err {err:.2e}")
    assert err <= 5e-4
    assert np.median(np.abs(g - rg) / (np.abs(rg) + 1e-6 * np.abs(rg).max())) <= 1e-5


def test_bf16_gradient_close_to_oracle():
    loss, per, g, rl, rp, rg, _ = run(4, 32, 48, 8, 2, "bf16", seed=2)
    cos = float(g @ rg / (np.linalg.norm(g) * np.linalg.norm(rg)))
    err = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"bf16 loss {loss:.5f} vs {rl:.5f}, grad cosine {cos:.5f}, rel err {err:.3e}")
    assert abs(loss - rl) <= 2e-2 * rl
    assert cos >= 0.99 and err <= 5e-2


def test_adam_step_and_autograd_function():
    from paper_2607_16906_amd import hz
    ops, gps, rs = batch(24, 4, 2, seed=3)
    specs = unet.layer_specs(3, 16, 5)
    theta0 = he_uniform(unet.init_shapes(specs), rng_for(14, 2, 3))
    net = hz.Net(3, 16, 5, theta0)
    r = to_dev(rs.astype(np.complex64), torch.complex64)
    th = torch.from_numpy(theta0.copy()).cuda().requires_grad_(True)
    loss = hz.physics_loss(th, net, gps, r, prec="fp32")
    loss.backward()
    _, _, grad = hz.loss_backward(net, gps, r, prec="fp32")
    assert torch.equal(th.grad, grad)
    # two Adam steps on the device against the oracle's Adam on the same gradients
    t = th.detach().clone()
    m = torch.zeros_like(t)
    v = torch.zeros_like(t)
    tr, mr, vr = theta0.astype(np.float64), np.zeros(t.numel()), np.zeros(t.numel())
    for step in (1, 2):
        _, _, g = hz.loss_backward(net, gps, r, prec="fp32")
        gn = to_np(g).astype(np.float64)
        hz.adam_step(net, t, m, v, g, step, lr=1e-3, clip=1.0)
        tr, mr, vr = oadam.adam_step(tr, gn, mr, vr, step, lr=1e-3, clip=1.0)
        assert np.max(np.abs(to_np(t) - tr)) <= 1e-6
    # the network now holds the updated weights
    z1 = net.apply(gps[0], r[0], prec="fp32")
    net2 = hz.Net(3, 16, 5, t)
    z2 = net2.apply(gps[0], r[0], prec="fp32")
    assert torch.equal(z1, z2)


def test_training_batch_full_grid_sampled():
    # the training workload's grid (128^2 + 16 PML) and network (4 levels, 32 channels) on a
    # 4-sample slice of the batch: loss and gradient against the oracle in FP32 mode
    from paper_2607_16906_amd import hz
    cs, rs = c3_batch(batch=4, step=0)
    ops, gps = [], []
    for c in cs:
        op, gp = make_pair(c, 16)
        ops.append(op)
        gps.append(gp)
    specs = unet.layer_specs(4, 32, 5)
    theta = he_uniform(unet.init_shapes(specs), rng_for(3, 2, 0))
    net = hz.Net(4, 32, 5, theta)
    r = to_dev(rs.astype(np.complex64), torch.complex64)
    loss, per, g = hz.loss_backward(net, gps, r, prec="fp32")
    rl, rp, rg = unet.loss_and_grad(theta.astype(np.float64), specs, ops, rs.astype(np.complex64).astype(np.complex128))
    assert abs(to_np(loss)[0] - rl) <= 1e-5 * rl
    assert np.linalg.norm(to_np(g) - rg) / np.linalg.norm(rg) <= 1e-4


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_recompute_bit_identical(prec):
    # activation checkpointing: the same loss and gradient bits as keeping every activation,
    # with a smaller workspace (4 levels, 32 channels, a ragged 44 x 44 padded grid, batch 3)
    from paper_2607_16906_amd import hz
    ops, gps, rs = batch(30, 6, 3, seed=4)
    specs = unet.layer_specs(4, 32, 5)
    theta = he_uniform(unet.init_shapes(specs), rng_for(14, 2, 4))
    net = hz.Net(4, 32, 5, theta)
    r = to_dev(rs.astype(np.complex64), torch.complex64)
    full = hz.train_workspace_bytes(net, gps[0], 3, prec)
    ckpt = hz.train_workspace_bytes(net, gps[0], 3, prec, recompute=True)
    print(f"{prec} workspace {full} -> {ckpt} bytes")
    assert ckpt < full
    a = hz.loss_backward(net, gps, r, prec=prec)
    b = hz.loss_backward(net, gps, r, prec=prec, recompute=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    if prec == "fp32":
        rl, _, rg = unet.loss_and_grad(theta.astype(np.float64), specs, ops, rs.astype(np.complex64).astype(np.complex128))
        assert abs(to_np(b[0])[0] - rl) <= 1e-5 * rl
        assert np.linalg.norm(to_np(b[2]) - rg) / np.linalg.norm(rg) <= 5e-4
