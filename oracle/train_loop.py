"""Oracle: the epoch-based training loop of the neural operator (Section 3.4, Tables 3 and 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper trains on a fixed set of random samples per data set for up to a maximal number of
epochs with Adam, batch size 32, gradient clipping at 1 and a learning rate that starts at 1e-3
and decreases to 1e-5 (Table 3), and keeps the epoch with the lowest validation loss (Table 5
lists the saved epoch and its validation loss). Readings where the paper is silent:

* schedule: cosine in the epoch index, lr(e) = lr_min + (lr0 - lr_min)(1 + cos(pi e / (E - 1))) / 2,
  constant within an epoch, so the first epoch runs at lr0 and the last at lr_min;
* visiting order: one permutation of the training set per epoch, given as an input; batches are
  consecutive runs of that order and the last one is shorter when the batch size does not divide
  the set;
* Adam's step counter runs over all batches of all epochs; clipping is of the global L2 norm;
* validation loss: the mean per-sample loss over the whole validation set after each epoch;
  the saved parameters are those after the first epoch that reaches the lowest validation loss.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from oracle import adam, unet


def cosine_lr(epoch: int, epochs: int, lr0: float = 1e-3, lr_min: float = 1e-5) -> float:
    """Learning rate of epoch ``epoch`` (0-based) of ``epochs``."""
    if epochs <= 1:
        return lr0
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + math.cos(math.pi * epoch / (epochs - 1)))


def batches(order, batch: int):
    """Consecutive runs of ``batch`` indices of ``order`` (the last one may be shorter)."""
    order = np.asarray(order)
    return [order[i:i + batch] for i in range(0, len(order), batch)]


def mean_loss(theta, specs, problems, rs, batch: int, squared=False, dtype=np.float64) -> float:
    """Mean per-sample loss over a whole set, evaluated in runs of ``batch`` samples."""
    total = 0.0
    for idx in batches(np.arange(len(problems)), batch):
        _, per, _ = unet.loss_and_grad(theta, specs, [problems[i] for i in idx], rs[idx], squared,
                                       dtype, need_grad=False)
        total += float(np.sum(per))
    return total / len(problems)


@dataclass
class TrainResult:
    theta_best: np.ndarray
    best_epoch: int
    best_val: float
    theta_last: np.ndarray
    train_loss: list = field(default_factory=list)   # batch-mean loss of every step
    val_loss: list = field(default_factory=list)     # validation loss after every epoch
    lr: list = field(default_factory=list)           # learning rate of every epoch


def train(theta0, specs, problems, rs, val_problems, val_rs, orders, *, batch: int,
          lr0: float = 1e-3, lr_min: float = 1e-5, clip: float = 1.0, squared: bool = False,
          dtype=np.float64) -> TrainResult:
    """Run len(orders) epochs; orders[e] is the visiting order of epoch e.

    problems / rs: the training set (one grid size; rs [S, ny, nx] complex residuals);
    val_problems / val_rs: the validation set.
    """
    epochs = len(orders)
    theta = np.asarray(theta0, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    res = TrainResult(theta.copy(), -1, math.inf, theta.copy())
    for e in range(epochs):
        lr = cosine_lr(e, epochs, lr0, lr_min)
        res.lr.append(lr)
        for idx in batches(orders[e], batch):
            loss, _, g = unet.loss_and_grad(theta.astype(dtype), specs, [problems[i] for i in idx],
                                            rs[idx], squared, dtype)
            t += 1
            theta, m, v = adam.adam_step(theta, np.asarray(g, np.float64), m, v, t, lr=lr, clip=clip)
            res.train_loss.append(float(loss))
        vl = mean_loss(theta.astype(dtype), specs, val_problems, val_rs, batch, squared, dtype)
        res.val_loss.append(vl)
        if vl < res.best_val:
            res.best_val, res.best_epoch, res.theta_best = vl, e, theta.copy()
    res.theta_last = theta
    return res
