"""Oracle: the Adam update used to train the neural operator (Section 3.4, Table 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Adam (Kingma and Ba) with bias correction: m <- b1 m + (1 - b1) g,
v <- b2 v + (1 - b2) g^2, theta <- theta - lr * mhat / (sqrt(vhat) + eps) with
mhat = m / (1 - b1^t), vhat = v / (1 - b2^t). The paper's clipping "value 1" is
read as a clip of the global L2 norm of the gradient to 1 (applied before the
update when ``clip`` is given).
"""
from __future__ import annotations

import numpy as np


def clip_global_norm(g, clip):
    nrm = float(np.linalg.norm(g))
    if clip is not None and nrm > clip:
        return g * (clip / nrm), nrm
    return g, nrm


def adam_step(theta, g, m, v, t: int, *, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8, clip=None):
    """One Adam step at step number t >= 1. Returns (theta, m, v) as new arrays."""
    g, _ = clip_global_norm(np.asarray(g, dtype=np.float64), clip)
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
