"""Train the U-Net neural operator with the oracle's loss, gradient and Adam (CPU, float32).

TEST INFRASTRUCTURE: calls only ``oracle`` and the input generators in ``synth``.
It writes the parameter file that the solver workloads load as their network
input, so that neither the oracle nor the GPU path ever consumes weights
produced by the GPU path.

Follows Sections 3.2-3.4: the physics-informed relative-residual loss (eq. (12),
unsquared by default), Adam with learning rate 1e-3 decaying to 1e-5, gradient
clipping at 1 and seed 42 (Table 3), single precision (Section 3.4), on a
mixture of velocity and source classes like dataset D0 (Table 4) with skull
rings standing in for the idealized skulls. Grids are small (the network is
fully convolutional and is applied to larger grids later, Section 4.2).

With --arch paper8 it trains Table 2's own layer set (oracle/unet8.py: --levels is the depth and
--base the channels per layer) instead of the 3x3 network.

Usage: python -m oracle.train_weights --out FILE [--steps N] [--batch B] [--levels L]
       [--base C] [--resume CKPT] [--ckpt CKPT] [--lr0 LR] [--restart STEP] [--arch unet3|paper8]
       [--dataset mix|D0..D5]
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

from oracle import adam, unet, unet8
from oracle import helmholtz as hz
from synth import C_REF, H_10PPW, he_uniform, mixed_training_sample, rng_for, table4_sample


def sample_batch(step: int, batch: int, nint: int, dataset: str = "mix"):
    """One batch: a PML width drawn per batch, a (velocity, source) pair per sample, from the
    D0-like mixture ("mix") or one of the data sets D0..D5 of Section 3.2 (Table 4)."""
    r = rng_for(42, 5, step)
    p = int(r.integers(12, 21))
    nt = nint + 2 * p
    problems, rs = [], []
    for s in range(batch):
        if dataset == "mix":
            c, b = mixed_training_sample(nt, p, rng_for(42, 6, step * batch + s))
        else:
            c, b = table4_sample(dataset, nt, p, rng_for(42, 10 + int(dataset[1]), step * batch + s))
        problems.append(hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF))
        rs.append(b)
    return problems, np.stack(rs)


def lr_at(step: int, total: int, lr0: float = 1e-3, lr_min: float = 1e-5, restart: int = 0) -> float:
    """Cosine decay from lr0 to lr_min over [restart, total) (restart > 0: a warm restart of the
    schedule for a continued run)."""
    span = max(total - restart, 1)
    k = min(max(step - restart, 0), span)
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * k / span))


def save(path, theta, specs, levels, base, in_ch, step, loss_hist, m=None, v=None, arch="unet3"):
    tmp = path + ".tmp.npz"
    extra = {} if m is None else {"adam_m": m, "adam_v": v}
    np.savez(tmp, theta=np.asarray(theta, np.float32), levels=levels, base=base, in_ch=in_ch,
             step=step, loss=np.asarray(loss_hist, np.float64), arch=arch, **extra)
    os.replace(tmp, path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--nint", type=int, default=64)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--in-ch", type=int, default=5)
    ap.add_argument("--save-every", type=int, default=100)
    ap.add_argument("--lr0", type=float, default=1e-3, help="peak learning rate of the cosine schedule")
    ap.add_argument("--restart", type=int, default=0, help="step at which the cosine schedule restarts")
    ap.add_argument("--arch", default="unet3", choices=["unet3", "paper8"])
    ap.add_argument("--dataset", default="mix", choices=["mix"] + [f"D{k}" for k in range(6)],
                    help="the D0-like mixture or a Table 4 data set")
    args = ap.parse_args()

    if args.arch == "paper8":
        net = unet8
        specs = unet8.layer_specs(args.levels, args.base, args.in_ch)
        theta = unet8.init_theta(specs, rng_for(42, 2, 0)).astype(np.float64)
    else:
        net = unet
        specs = unet.layer_specs(args.levels, args.base, args.in_ch)
        theta = he_uniform(unet.init_shapes(specs), rng_for(42, 2, 0)).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    start, hist = 0, []
    if args.resume and os.path.exists(args.resume):
        ck = np.load(args.resume)
        theta = ck["theta"].astype(np.float64)
        m, v = ck["adam_m"], ck["adam_v"]
        start, hist = int(ck["step"]), list(ck["loss"])
        print(f"resumed at step {start}", flush=True)
    t0 = time.time()
    for step in range(start, args.steps):
        problems, rs = sample_batch(step, args.batch, args.nint, args.dataset)
        loss, _, g = net.loss_and_grad(theta.astype(np.float32), specs, problems, rs, dtype=np.float32)
        theta, m, v = adam.adam_step(theta, g.astype(np.float64), m, v, step + 1,
                                     lr=lr_at(step, args.steps, args.lr0, restart=args.restart), clip=1.0)
        hist.append(loss)
        if (step + 1) % 10 == 0:
            print(f"step {step + 1} loss {np.mean(hist[-10:]):.4f} "
                  f"lr {lr_at(step, args.steps, args.lr0, restart=args.restart):.2e} "
                  f"{(time.time() - t0) / (step + 1 - start):.2f} s/step", flush=True)
        if (step + 1) % args.save_every == 0 or step + 1 == args.steps:
            save(args.out, theta, specs, args.levels, args.base, args.in_ch, step + 1, hist, arch=args.arch)
            if args.ckpt:
                save(args.ckpt, theta, specs, args.levels, args.base, args.in_ch, step + 1, hist, m, v,
                     arch=args.arch)


if __name__ == "__main__":
    main()
