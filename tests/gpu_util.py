"""Helpers shared by the GPU parity tests: build matching oracle and GPU problems from one
seeded input, and move fields between numpy and the device."""
import numpy as np

from oracle import helmholtz as ohz
from synth import C_REF, H_10PPW


def make_pair(c, npml, h=H_10PPW, omega=1.0, sigma_max=2.0):
    """(oracle Problem, GPU Problem) for the velocity field c [nt, nt] (m/s)."""
    from paper_2607_16906_amd import hz
    c = np.asarray(c, dtype=np.float32)          # the library takes FP32 velocities
    ny, nx = c.shape
    op = ohz.Problem(c.astype(np.float64), npml, h, omega, sigma_max, C_REF)
    gp = hz.Problem(c.ravel(), nx - 2 * npml, ny - 2 * npml, npml, h, omega, sigma_max, C_REF)
    return op, gp


def to_dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).ravel())).to(dtype).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
