"""Pins of the oracle's Adam update (Section 3.4, Table 3): the closed form of the first step and
agreement with torch.optim.Adam over several steps."""
import numpy as np
import torch

from oracle import adam


def test_first_step_closed_form():
    # at t = 1 the bias-corrected moments are g and g^2, so the step is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    th, m, v = adam.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)


def test_matches_torch_adam():
    rng = np.random.default_rng(0)
    th0 = rng.standard_normal(50)
    p = torch.tensor(th0.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g.copy())
        opt.step()
        th, m, v = adam.adam_step(th, g, m, v, t, lr=1e-2)
    assert np.max(np.abs(th - p.detach().numpy())) < 1e-13


def test_global_norm_clip():
    g = np.array([3.0, 4.0])
    gc, n = adam.clip_global_norm(g, 1.0)
    assert n == 5.0 and np.allclose(gc, [0.6, 0.8])
    gc, _ = adam.clip_global_norm(np.array([0.3, 0.4]), 1.0)
    assert np.allclose(gc, [0.3, 0.4])
