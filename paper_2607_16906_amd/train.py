"""Epoch-based training of the neural operator on the GPU (Section 3.4, Tables 3 and 5).

Host orchestration over the library's entry points: every step of a batch runs in the library
(no_loss_backward for the loss of eq. (12) and its gradient, no_adam_step for the clipped Adam
update); this module only chooses the batches, the learning rate of each epoch and the saved
epoch. The data set stays resident on the device for the whole run: one problem handle per
sample and the residuals as one [S, n] complex64 tensor, gathered per batch in the epoch's order.

Schedule and selection (the paper gives the end points and the saved-epoch rule only):
* the learning rate is constant within an epoch and follows a cosine in the epoch index from
  lr0 (first epoch) to lr_min (last epoch), 1e-3 and 1e-5 by default (Table 3);
* each epoch visits the training set once, in the order given for it, in batches of ``batch``
  samples (the last batch is shorter when ``batch`` does not divide the set);
* Adam's step counter runs over all batches; the gradient is clipped to global L2 norm ``clip``;
* after each epoch the validation loss (the mean per-sample loss over the validation set, a
  forward-only pass) is computed, and the parameters of the first epoch with the lowest
  validation loss are kept (Table 5 lists the saved epoch and its validation loss).
"""
from __future__ import annotations

import ctypes as ct
import math
from dataclasses import dataclass, field

import numpy as np

from . import hz


def cosine_lr(epoch: int, epochs: int, lr0: float = 1e-3, lr_min: float = 1e-5) -> float:
    """Learning rate of epoch ``epoch`` (0-based) of ``epochs``."""
    if epochs <= 1:
        return lr0
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * epoch / (epochs - 1)))


@dataclass
class FitResult:
    theta_best: object                               # device float32 [nparam]
    best_epoch: int
    best_val: float
    theta_last: object                               # device float32 [nparam]
    train_loss: np.ndarray = None                    # batch-mean loss of every step
    val_loss: list = field(default_factory=list)     # validation loss after every epoch
    lr: list = field(default_factory=list)           # learning rate of every epoch
    step_ms: float = 0.0                             # mean wall time of a training step
    val_ms: float = 0.0                              # mean wall time of a validation pass


class Trainer:
    """Runs epochs of training for one network on one resident data set.

    net: hz.Net; problems / val_problems: hz.Problem lists of one grid size;
    r / val_r: [S, n] / [V, n] complex64 device tensors (the sources, used as residuals).
    """

    def __init__(self, net: hz.Net, problems, r, val_problems, val_r, *, batch: int = 32,
                 prec: str = "bf16", squared: bool = False, recompute: bool = False):
        torch = hz._torch()
        self.lib = hz.load_library()
        self.net, self.batch, self.prec = net, int(batch), prec
        self.squared, self.recompute = int(squared), int(recompute)
        self.problems, self.val_problems = list(problems), list(val_problems)
        S, V = len(self.problems), len(self.val_problems)
        if S < 1 or V < 1 or self.batch < 1:
            raise ValueError("need at least one training sample, one validation sample and batch >= 1")
        p0 = self.problems[0]
        for p in self.problems + self.val_problems:
            if (p.nxt, p.nyt, p.npml) != (p0.nxt, p0.nyt, p0.npml):
                raise ValueError("every sample must have the same grid and PML")
        self.n = p0.n
        if tuple(r.shape) != (S, self.n) or tuple(val_r.shape) != (V, self.n):
            raise ValueError("r must be [S, n] and val_r [V, n]")
        if r.dtype != torch.complex64 or val_r.dtype != torch.complex64 or not r.is_cuda or not val_r.is_cuda:
            raise ValueError("r and val_r must be complex64 device tensors")
        self.r, self.val_r = r.contiguous(), val_r.contiguous()
        self.handles = np.array([p.handle.value for p in self.problems], dtype=np.uint64)
        self.val_handles = np.array([p.handle.value for p in self.val_problems], dtype=np.uint64)
        # workspace for the largest batch (the training workspace grows with the batch)
        nb = max(self.lib.no_train_workspace_size(net.handle, p0.handle, b, hz.PREC[prec], self.recompute)
                 for b in {min(self.batch, S), min(self.batch, V)})
        self.ws = hz._ws(nb)
        self.aws = hz._ws(self.lib.no_adam_workspace_size(net.handle))
        self.grad = torch.empty(net.nparam, dtype=torch.float32, device="cuda")
        self.rb = torch.empty((min(self.batch, S), self.n), dtype=torch.complex64, device="cuda")
        self.per = torch.empty(max(min(self.batch, S), V), dtype=torch.float32, device="cuda")
        self.vloss = torch.empty(1, dtype=torch.float32, device="cuda")

    def _loss(self, handles, rptr, bsz, loss_ptr, per_ptr, grad):
        ptrs = (ct.c_void_p * bsz)(*[int(h) for h in handles])
        hz._check(self.lib.no_loss_backward(self.net.handle, bsz, ptrs, ct.c_void_p(rptr), self.squared,
                                            self.recompute, hz.PREC[self.prec], ct.c_void_p(loss_ptr),
                                            ct.c_void_p(per_ptr), hz._ptr(grad) if grad is not None else None,
                                            hz._ptr(self.ws), ct.c_size_t(self.ws.numel()), hz._stream()),
                  "no_loss_backward")

    def validation_loss(self) -> float:
        """Mean per-sample loss over the validation set at the network's current weights."""
        V = len(self.val_problems)
        for i in range(0, V, self.batch):
            bsz = min(self.batch, V - i)
            self._loss(self.val_handles[i:i + bsz], self.val_r.data_ptr() + 8 * self.n * i, bsz,
                       self.vloss.data_ptr(), self.per.data_ptr() + 4 * i, None)
        per = self.per[:V].cpu().numpy().astype(np.float64)    # synchronises the stream
        return float(per.sum() / V)

    def fit(self, theta0, orders, *, lr0: float = 1e-3, lr_min: float = 1e-5, clip: float = 1.0,
            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, log=None) -> FitResult:
        """Train for len(orders) epochs from theta0 (orders[e]: the visiting order of epoch e)."""
        import time
        torch = hz._torch()
        S, E = len(self.problems), len(orders)
        theta = torch.as_tensor(theta0, dtype=torch.float32).to("cuda").clone().contiguous()
        if theta.numel() != self.net.nparam:
            raise ValueError("theta0 does not match the network")
        m = torch.zeros_like(theta)
        v = torch.zeros_like(theta)
        self.net.set_weights(theta)
        steps_per_epoch = (S + self.batch - 1) // self.batch
        losses = torch.empty(E * steps_per_epoch, dtype=torch.float32, device="cuda")
        res = FitResult(theta.clone(), -1, math.inf, theta)
        t, tstep, tval = 0, 0.0, 0.0
        for e in range(E):
            order = np.asarray(orders[e], dtype=np.int64)
            if order.shape != (S,) or not np.array_equal(np.sort(order), np.arange(S)):
                raise ValueError(f"orders[{e}] is not a permutation of the training set")
            lr = cosine_lr(e, E, lr0, lr_min)
            res.lr.append(lr)
            idx = torch.from_numpy(order).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(0, S, self.batch):
                bsz = min(self.batch, S - i)
                torch.index_select(self.r, 0, idx[i:i + bsz], out=self.rb[:bsz])
                self._loss(self.handles[order[i:i + bsz]], self.rb.data_ptr(), bsz,
                           losses.data_ptr() + 4 * t, self.per.data_ptr(), self.grad)
                t += 1
                hz._check(self.lib.no_adam_step(self.net.handle, hz._ptr(theta), hz._ptr(m), hz._ptr(v),
                                                hz._ptr(self.grad), t, lr, beta1, beta2, eps, clip,
                                                hz._ptr(self.aws), ct.c_size_t(self.aws.numel()), hz._stream()),
                          "no_adam_step")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            vl = self.validation_loss()
            tval += time.perf_counter() - t1
            tstep += t1 - t0
            res.val_loss.append(vl)
            if vl < res.best_val:
                res.best_val, res.best_epoch = vl, e
                res.theta_best.copy_(theta)
            if log:
                tl = losses[t - steps_per_epoch:t].cpu().numpy().astype(np.float64).mean()
                log(f"epoch {e} lr {lr:.2e} train {tl:.4f} val {vl:.4f}")
        res.theta_last = theta
        res.train_loss = losses[:t].cpu().numpy().astype(np.float64)
        res.step_ms = 1e3 * tstep / max(t, 1)
        res.val_ms = 1e3 * tval / max(E, 1)
        return res


def resident_set(c, b, nint: int, npml: int, h: float, disc: str = "fd"):
    """Upload a data set: velocities c [S, nt, nt] (m/s) and sources b [S, nt, nt] (complex) to one
    hz.Problem per sample (discretization disc: "fd" or "spectral") and one [S, n] complex64
    device tensor."""
    torch = hz._torch()
    probs = [hz.Problem(ci.astype(np.float32).ravel(), nint, nint, npml, h, disc=disc) for ci in c]
    r = torch.from_numpy(np.ascontiguousarray(b.reshape(len(b), -1)).astype(np.complex64)).to("cuda")
    return probs, r


def save_weights(path, theta, *, levels, base, in_ch, dataset, nint, npml, epochs, best_epoch, best_val, steps,
                 bf16=False, arch="unet3", disc="fd"):
    """Write a parameter file: float32 theta (or, bf16=True, its BF16 rounding as 16-bit patterns,
    half the size, for networks that only run with BF16 operands) and the training record."""
    th = np.asarray(theta, np.float32)
    rec = dict(levels=levels, base=base, in_ch=in_ch, dataset=dataset, nint=nint, npml=npml, epochs=epochs,
               best_epoch=best_epoch, best_val=best_val, step=steps, arch=arch, disc=disc)
    if bf16:
        u = th.view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
        np.savez(path, theta_bf16=u, **rec)
    else:
        np.savez(path, theta=th, **rec)


def load_weights(path):
    """theta (float32) of a parameter file written by save_weights (or by the oracle's trainer)."""
    w = np.load(path)
    if "theta" in w:
        return w["theta"].astype(np.float32)
    return (w["theta_bf16"].astype(np.uint32) << 16).view(np.float32)


def init_theta_paper8(depth: int, ch: int, in_ch: int, rng, slope: float = 0.25) -> np.ndarray:
    """Seeded He-uniform weights and biases of Table 2's network (hz.init_shapes_paper8 order), each
    layer but the 1x1 head followed by its PReLU slope (0.25, the usual PReLU initial value)."""
    from synth import he_uniform
    shapes = hz.init_shapes_paper8(depth, ch, in_ch)
    parts = []
    for i, sh in enumerate(shapes):
        parts.append(he_uniform([sh], rng))
        if i + 1 < len(shapes):
            parts.append(np.array([slope], np.float32))
    return np.concatenate(parts).astype(np.float32)


def main():
    """Train a network on one of the Table 4 data sets on the GPU and write its parameter file:
    the 3x3 U-Net (--arch unet3; --levels, --base) or Table 2's 8x8 stride-2 network with PReLU
    (--arch paper8; --levels is its depth, --base its channels per layer; FP32, as Section 3.4).

    Usage: python -m paper_2607_16906_amd.train --out FILE [--arch unet3] [--dataset D0] [--levels 5]
           [--base 32] [--nint 128] [--npml 16] [--count 4096] [--val 256] [--epochs 24] [--batch 32]
           [--prec fp32] [--bf16-file] [--disc fd|spectral]
    """
    import argparse
    import time

    import torch

    from synth import (CFG_TABLE4, COMP_ORDER, COMP_WEIGHTS, H_10PPW, VAL_FIRST, he_uniform, rng_for,
                       table4_set, training_set)
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--arch", default="unet3", choices=["unet3", "paper8"])
    ap.add_argument("--dataset", default="D0", choices=[f"D{k}" for k in range(6)] + ["mix"],
                    help="a Table 4 data set, or 'mix': the D0-like mixture with smooth source classes "
                         "(Gaussian blobs, box-smoothed noise) beside the paper's ones")
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--nint", type=int, default=128)
    ap.add_argument("--npml", type=int, default=16)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--val", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=24)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--bf16-file", action="store_true", help="store the BF16 rounding of the weights")
    ap.add_argument("--disc", default="fd", choices=["fd", "spectral"],
                    help="operator of the loss: finite differences or Fourier differentiation (Section 2.1)")
    a = ap.parse_args()
    if a.arch == "paper8" and a.prec != "fp32":
        ap.error("the paper8 network trains in FP32")
    torch.cuda.set_device(0)
    nt = a.nint + 2 * a.npml
    t0 = time.time()
    if a.dataset == "mix":
        c, b = training_set(a.count, nt, a.npml)
        cv, bv = training_set(a.val, nt, a.npml, first=VAL_FIRST)
    else:
        c, b = table4_set(a.dataset, a.count, nt, a.npml)
        cv, bv = table4_set(a.dataset, a.val, nt, a.npml, first=VAL_FIRST)
    probs, r = resident_set(c, b, a.nint, a.npml, H_10PPW, a.disc)
    vprobs, vr = resident_set(cv, bv, a.nint, a.npml, H_10PPW, a.disc)
    print(f"data set {a.dataset}: {a.count} + {a.val} samples on {nt}^2 in {time.time() - t0:.1f} s", flush=True)
    if a.arch == "paper8":
        theta0 = init_theta_paper8(a.levels, a.base, 5, rng_for(CFG_TABLE4, COMP_WEIGHTS, 100 + a.levels))
    else:
        theta0 = he_uniform(hz.init_shapes(a.levels, a.base, 5), rng_for(CFG_TABLE4, COMP_WEIGHTS, a.levels))
    net = hz.Net(a.levels, a.base, 5, theta0, kind=a.arch)
    tr = Trainer(net, probs, r, vprobs, vr, batch=a.batch, prec=a.prec)
    orders = [rng_for(CFG_TABLE4, COMP_ORDER, e).permutation(a.count) for e in range(a.epochs)]
    res = tr.fit(theta0, orders, log=lambda msg: print(msg, flush=True))
    steps = a.epochs * ((a.count + a.batch - 1) // a.batch)
    print(f"best epoch {res.best_epoch} val {res.best_val:.4f}; {steps} steps, {res.step_ms:.2f} ms per step",
          flush=True)
    save_weights(a.out, res.theta_best.cpu().numpy(), levels=a.levels, base=a.base, in_ch=5, dataset=a.dataset,
                 nint=a.nint, npml=a.npml, epochs=a.epochs, best_epoch=res.best_epoch, best_val=res.best_val,
                 steps=steps, bf16=a.bf16_file, arch=a.arch, disc=a.disc)


if __name__ == "__main__":
    main()
