"""Pins of the oracle's epoch-based training loop (Section 3.4, Tables 3 and 5).

The loop is checked against an independent statement built from torch's own optimizer, scheduler
and autograd (torch.optim.Adam, CosineAnnealingLR stepped once per epoch, dense operators), and
against properties that any correct loop has: zero learning rate leaves the parameters alone, the
saved parameters reproduce the saved validation loss, and training lowers the validation loss.
"""
import math

import numpy as np
import torch
import torch.nn.functional as F

from oracle import helmholtz as hz
from oracle import train_loop, unet
from synth import (C_REF, H_10PPW, box_smoothed_noise, epoch_order, he_uniform, rng_for,
                   skull_ring_velocity, training_set)


def test_cosine_schedule_matches_torch_scheduler():
    for epochs in (2, 5, 17):
        p = torch.nn.Parameter(torch.zeros(1))
        opt = torch.optim.SGD([p], lr=1e-3)
        sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=epochs - 1, eta_min=1e-5)
        for e in range(epochs):
            assert abs(opt.param_groups[0]["lr"] - train_loop.cosine_lr(e, epochs)) <= 1e-15
            opt.step()
            sch.step()
    # the paper's end points: it starts at 1e-3 and decreases to 1e-5
    assert train_loop.cosine_lr(0, 500) == 1e-3 and abs(train_loop.cosine_lr(499, 500) - 1e-5) < 1e-18


def test_batches_cover_the_order_once():
    order = epoch_order(10, 3)
    bs = train_loop.batches(order, 4)
    assert [len(b) for b in bs] == [4, 4, 2]
    assert np.array_equal(np.concatenate(bs), order)
    assert sorted(order.tolist()) == list(range(10))


def small_set(count, first, nx=24, p=4):
    nt = nx + 2 * p
    probs, rs = [], []
    for i in range(count):
        c = skull_ring_velocity(nt, p, rng_for(9, 0, first + i), rings=1)
        probs.append(hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF))
        rs.append(box_smoothed_noise(nt, rng_for(9, 3, first + i)))
    return probs, np.stack(rs)


def torch_loss(th, specs, problems, rs, levels):
    """The unsquared batch-mean loss stated with torch.nn.functional and dense operators."""
    P, off = {}, 0
    for name, kind, ci, co in specs:
        shp = unet.weight_shape(kind, ci, co)
        nw = int(np.prod(shp))
        P[name] = (th[off:off + nw].reshape(shp), th[off + nw:off + nw + co])
        off += nw + co
    total = 0
    for b, p in enumerate(problems):
        r = rs[b]
        s = np.linalg.norm(r) / np.sqrt(r.size)
        sx, sy = p.sigma_nodes()
        h = torch.tensor(np.stack([r.real / s, r.imag / s, p.c / p.c_ref, sx, sy])[None])
        skips = []
        for l in range(levels):
            if l:
                h = F.avg_pool2d(h, 2)
            h = F.relu(F.conv2d(h, *P[f"enc{l}a"], padding=1))
            h = F.relu(F.conv2d(h, *P[f"enc{l}b"], padding=1))
            skips.append(h)
        for l in range(levels - 2, -1, -1):
            u = F.conv_transpose2d(h, *P[f"up{l}"], stride=2)
            h = torch.cat([skips[l], u], 1)
            h = F.relu(F.conv2d(h, *P[f"dec{l}a"], padding=1))
            h = F.relu(F.conv2d(h, *P[f"dec{l}b"], padding=1))
        out = F.conv2d(h, *P["head"])[0]
        z = s * torch.complex(out[0], out[1]).reshape(-1)
        q = torch.tensor(hz.assemble_dense(p)) @ z - torch.tensor(r.ravel())
        total = total + torch.linalg.vector_norm(q) / np.linalg.norm(r)
    return total / len(problems)


def test_loop_matches_torch_optimizer_loop():
    levels, base = 2, 4
    specs = unet.layer_specs(levels, base, 5)
    theta0 = he_uniform(unet.init_shapes(specs), np.random.default_rng(3)).astype(np.float64)
    probs, rs = small_set(5, 0)
    vprobs, vrs = small_set(2, 100)
    epochs, batch = 3, 2
    orders = [epoch_order(5, e) for e in range(epochs)]
    res = train_loop.train(theta0, specs, probs, rs, vprobs, vrs, orders, batch=batch, lr0=1e-2,
                           lr_min=1e-4, clip=1e30)
    # the same loop with torch's Adam, its cosine scheduler and autograd
    th = torch.tensor(theta0.copy(), requires_grad=True)
    opt = torch.optim.Adam([th], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=epochs - 1, eta_min=1e-4)
    tl, vl, best = [], [], (math.inf, -1, None)
    for e in range(epochs):
        order = orders[e]
        for i in range(0, len(order), batch):
            idx = order[i:i + batch]
            opt.zero_grad()
            loss = torch_loss(th, specs, [probs[j] for j in idx], rs[idx], levels)
            loss.backward()
            opt.step()
            tl.append(loss.item())
        with torch.no_grad():
            v = sum(torch_loss(th, specs, [vprobs[j]], vrs[[j]], levels).item() for j in range(2)) / 2
        vl.append(v)
        if v < best[0]:
            best = (v, e, th.detach().numpy().copy())
        sch.step()
    assert len(res.train_loss) == epochs * 3
    assert np.allclose(res.train_loss, tl, rtol=1e-11, atol=0)
    assert np.allclose(res.val_loss, vl, rtol=1e-11, atol=0)
    assert res.best_epoch == best[1]
    assert np.max(np.abs(res.theta_last - th.detach().numpy())) <= 1e-10
    assert np.max(np.abs(res.theta_best - best[2])) <= 1e-10


def test_zero_rate_keeps_parameters_and_first_minimum_is_saved():
    specs = unet.layer_specs(2, 4, 5)
    theta0 = he_uniform(unet.init_shapes(specs), np.random.default_rng(4)).astype(np.float64)
    probs, rs = small_set(3, 10)
    vprobs, vrs = small_set(2, 110)
    res = train_loop.train(theta0, specs, probs, rs, vprobs, vrs, [epoch_order(3, e) for e in range(2)],
                           batch=2, lr0=0.0, lr_min=0.0)
    assert np.array_equal(res.theta_last, theta0) and np.array_equal(res.theta_best, theta0)
    assert res.val_loss[0] == res.val_loss[1] and res.best_epoch == 0


def test_training_lowers_validation_loss_and_saved_parameters_reproduce_it():
    # the D0-like mixture on a 24^2 + 4 PML grid, 4-level / 4-channel network
    nt, p = 32, 4
    specs = unet.layer_specs(3, 4, 5)
    theta0 = he_uniform(unet.init_shapes(specs), rng_for(42, 2, 0)).astype(np.float64)
    c, b = training_set(8, nt, p)
    vc, vb = training_set(4, nt, p, first=10_000_000)
    mk = lambda cs: [hz.Problem(ci, p, H_10PPW, 1.0, 2.0, C_REF) for ci in cs]
    probs, vprobs = mk(c), mk(vc)
    res = train_loop.train(theta0, specs, probs, b, vprobs, vb, [epoch_order(8, e) for e in range(4)],
                           batch=4, lr0=1e-2, lr_min=1e-3)
    v0 = train_loop.mean_loss(theta0, specs, vprobs, vb, 4)
    assert res.best_val < 0.9 * v0
    assert res.best_epoch == int(np.argmin(res.val_loss))
    assert abs(train_loop.mean_loss(res.theta_best, specs, vprobs, vb, 3) - res.best_val) <= 1e-12 * res.best_val
