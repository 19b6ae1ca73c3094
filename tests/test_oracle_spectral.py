"""Pins of the oracle's Fourier-differentiation operator, none of which goes through its FFT code:
the closed-form periodic differentiation matrix (the cot / csc entries of the derivative of the
periodic sinc interpolant) fixes the wavenumber scaling, sign and Nyquist treatment; exact Fourier
eigenmodes (no PML) fix the assembly of both axes and the k^2 term; the derivative of a smooth
periodic function to near rounding fixes the spectral accuracy; a PML-aware dense matrix written
from the closed-form matrix fixes the stretching order, and the dot test fixes the adjoint."""
import math

import numpy as np
import pytest

from oracle import helmholtz as hz
from oracle import spectral as sp
from synth import C_REF, H_10PPW, rng_for, skull_ring_velocity


def diff_matrix(n, h):
    """Periodic spectral differentiation matrix from its closed form: for j != l,
    D[j, l] = (pi / L) (-1)^(j-l) cot(pi (j - l) / n) (n even) or csc(...) (n odd), L = n h."""
    L = n * h
    D = np.zeros((n, n))
    for j in range(n):
        for l in range(n):
            if j != l:
                t = math.pi * (j - l) / n
                f = 1.0 / math.tan(t) if n % 2 == 0 else 1.0 / math.sin(t)
                D[j, l] = (math.pi / L) * (-1) ** (j - l) * f
    return D


@pytest.mark.parametrize("n", [8, 9, 16, 23, 40])
def test_derivative_matches_closed_form_matrix(n):
    h = 0.37
    D = diff_matrix(n, h)
    cols = np.stack([sp.deriv(np.eye(n)[:, l], 0, h) for l in range(n)], axis=1)
    assert np.max(np.abs(cols.imag)) <= 1e-13 * np.max(np.abs(D))
    assert np.max(np.abs(cols.real - D)) <= 1e-12 * np.max(np.abs(D))
    assert np.max(np.abs(D + D.T)) == 0.0   # antisymmetric (the adjoint's premise)


def test_derivative_spectral_accuracy():
    # f = exp(sin(2 pi x / L)) is periodic and entire: its derivative is reproduced to near rounding
    n, h = 64, 0.2
    L = n * h
    x = np.arange(n) * h
    f = np.exp(np.sin(2 * np.pi * x / L))
    df = (2 * np.pi / L) * np.cos(2 * np.pi * x / L) * f
    assert np.max(np.abs(sp.deriv(f, 0, h) - df)) <= 1e-11 * np.max(np.abs(df))


@pytest.mark.parametrize("mx,my", [(0, 0), (1, 2), (5, -3), (-7, 9)])
def test_fourier_eigenmodes(mx, my):
    # no PML, constant c: exp(i kx x) exp(i ky y) (|m| < n/2) has eigenvalue k^2 - kx^2 - ky^2
    nx, ny = 24, 20
    P = hz.Problem(np.full((ny, nx), 1.2 * C_REF), 0, H_10PPW, 1.0, 0.0, C_REF)
    kx = 2 * np.pi * mx / (nx * P.h)
    ky = 2 * np.pi * my / (ny * P.h)
    x = np.arange(nx) * P.h
    y = np.arange(ny) * P.h
    u = np.outer(np.exp(1j * ky * y), np.exp(1j * kx * x))
    lam = (1 / 1.2) ** 2 - kx ** 2 - ky ** 2
    assert np.max(np.abs(sp.op_apply(P, u) - lam * u)) <= 1e-12 * (abs(lam) + 1)


def dense_operator(P):
    """A as a dense matrix built from the closed-form D and the node stretching (row-major index)."""
    Dx, Dy = diff_matrix(P.nx, P.h), diff_matrix(P.ny, P.h)
    gx = np.diag(sp.inv_gamma(P.nx, P.npml, P.omega, P.sigma_max))
    gy = np.diag(sp.inv_gamma(P.ny, P.npml, P.omega, P.sigma_max))
    Mx = gx @ Dx @ gx @ Dx
    My = gy @ Dy @ gy @ Dy
    A = np.kron(np.eye(P.ny), Mx) + np.kron(My, np.eye(P.nx)) + np.diag(P.k2.ravel())
    return A


def test_dense_operator_with_pml_and_adjoint():
    nt, p = 18, 4
    c = skull_ring_velocity(nt, p, rng_for(30, 0, 0), rings=1)
    P = hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF)
    A = dense_operator(P)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt))
    w = rng.standard_normal((nt, nt)) + 1j * rng.standard_normal((nt, nt))
    Au = sp.op_apply(P, u).ravel()
    assert np.linalg.norm(Au - A @ u.ravel()) <= 1e-12 * np.linalg.norm(Au)
    AHw = sp.op_adjoint(P, w).ravel()
    assert np.linalg.norm(AHw - A.conj().T @ w.ravel()) <= 1e-12 * np.linalg.norm(AHw)
    # dot test
    lhs = np.vdot(Au, w.ravel())
    rhs = np.vdot(u.ravel(), AHw)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
