"""Oracle: the Fourier-differentiation (pseudo-spectral) form of the 2-D Helmholtz operator with
a PML, the discretization the paper itself computes (Section 2.1 and Table 1: derivatives by the
FFT over both grid axes, which makes the grid periodic).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid, wavenumber and PML damping are those of helmholtz.py: nodes i = 0..N-1 per axis with
spacing h, sigma(i) = sigma_max (depth / npml)^2 at the nodes, stretch gamma = 1 + i sigma / omega.

Spectral first derivative of a periodic grid function f of N nodes along one axis:
    D f = IFFT( i kappa FFT(f) ),
    kappa_m = 2 pi m / (N h) for m < N / 2 and 2 pi (m - N) / (N h) for m > N / 2,
with kappa = 0 at the Nyquist index m = N / 2 when N is even (the sampled derivative of that mode
vanishes at the nodes; zeroing it keeps D real and antisymmetric).

Operator (complex coordinate stretching d/dx -> (1 / gamma) d/dx on each axis):
    A u   = (1/gx) Dx((1/gx) Dx u) + (1/gy) Dy((1/gy) Dy u) + k^2 u,
and, since D^T = -D and k^2 is real,
    A^H w = Dx(conj(1/gx) Dx(conj(1/gx) w)) + Dy(conj(1/gy) Dy(conj(1/gy) w)) + k^2 w.
A grid vector has shape [ny, nx] (flattened index j * nx + i), as in helmholtz.py.
"""
from __future__ import annotations

import numpy as np

from .helmholtz import Problem, pml_sigma  # noqa: F401  (Problem: the same grid / k^2 holder)


def wavenumbers(n: int, h: float) -> np.ndarray:
    """kappa_m in FFT order, with the Nyquist entry of an even n set to 0."""
    m = np.arange(n, dtype=np.float64)
    m = np.where(m < n / 2, m, m - n)
    kap = 2.0 * np.pi * m / (n * h)
    if n % 2 == 0:
        kap[n // 2] = 0.0
    return kap


def deriv(f, axis: int, h: float):
    """Spectral first derivative of the periodic grid function f along `axis`."""
    f = np.asarray(f, dtype=np.complex128)
    n = f.shape[axis]
    shape = [1] * f.ndim
    shape[axis] = n
    ik = (1j * wavenumbers(n, h)).reshape(shape)
    return np.fft.ifft(ik * np.fft.fft(f, axis=axis), axis=axis)


def inv_gamma(n: int, npml: int, omega: float, sigma_max: float) -> np.ndarray:
    """1 / gamma at the nodes of one axis, complex128 [n]."""
    return 1.0 / (1.0 + 1j * pml_sigma(np.arange(n), n, npml, sigma_max) / omega)


def op_apply(op: Problem, u):
    """A u for one grid vector u [ny, nx] (complex)."""
    u = np.asarray(u, dtype=np.complex128)
    gx = inv_gamma(op.nx, op.npml, op.omega, op.sigma_max)[None, :]
    gy = inv_gamma(op.ny, op.npml, op.omega, op.sigma_max)[:, None]
    ax = gx * deriv(gx * deriv(u, 1, op.h), 1, op.h)
    ay = gy * deriv(gy * deriv(u, 0, op.h), 0, op.h)
    return ax + ay + op.k2 * u


def op_adjoint(op: Problem, w):
    """A^H w for one grid vector w [ny, nx] (complex)."""
    w = np.asarray(w, dtype=np.complex128)
    gx = np.conj(inv_gamma(op.nx, op.npml, op.omega, op.sigma_max))[None, :]
    gy = np.conj(inv_gamma(op.ny, op.npml, op.omega, op.sigma_max))[:, None]
    ax = deriv(gx * deriv(gx * w, 1, op.h), 1, op.h)
    ay = deriv(gy * deriv(gy * w, 0, op.h), 0, op.h)
    return ax + ay + op.k2 * w
