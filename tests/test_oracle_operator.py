"""Pins of the oracle's Helmholtz operator against closed forms and independent constructions.

Each check fixes something a plausible mistake would break: the Dirichlet sine
modes fix the Laplacian's scaling and boundary; the plane-wave dispersion fixes
the stencil's neighbour coupling and k^2 term; the dense assembly is written
entry by entry, independently of the vectorized apply; the free-space Green's
function (Hankel function) fixes the PML's sign and placement; the dot test fixes
the adjoint.
"""
import math

import numpy as np
import pytest
from scipy import optimize, special

from oracle import helmholtz as hz
from synth import C_REF, H_10PPW, c1_system


def homogeneous_problem(nx, ny, npml=0, sigma_max=0.0, c=C_REF, h=H_10PPW):
    return hz.Problem(np.full((ny, nx), c), npml, h, 1.0, sigma_max, C_REF)


@pytest.mark.parametrize("p,q", [(1, 1), (2, 5), (7, 3), (11, 11)])
def test_dirichlet_sine_eigenmodes(p, q):
    # With no PML and constant k, the five-point operator with zero values outside the grid has
    # eigenvectors sin(p pi (i+1)/(Nx+1)) sin(q pi (j+1)/(Ny+1)) and eigenvalues
    # k^2 - (4/h^2) [sin^2(p pi / (2(Nx+1))) + sin^2(q pi / (2(Ny+1)))].
    nx, ny = 13, 17
    P = homogeneous_problem(nx, ny, c=1.3 * C_REF)
    i = np.arange(nx)
    j = np.arange(ny)
    u = np.outer(np.sin(q * math.pi * (j + 1) / (ny + 1)), np.sin(p * math.pi * (i + 1) / (nx + 1)))
    k2 = (1.0 / 1.3) ** 2
    lam = k2 - 4.0 / P.h ** 2 * (math.sin(p * math.pi / (2 * (nx + 1))) ** 2
                                  + math.sin(q * math.pi / (2 * (ny + 1))) ** 2)
    Au = hz.op_apply(P, u)
    scale = 8.0 / P.h ** 2 + k2
    assert np.max(np.abs(Au - lam * u)) <= 1e-12 * scale


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, math.pi / 4])
def test_plane_wave_discrete_dispersion(theta):
    # exp(i kappa (x cos t + y sin t)) is annihilated at every node away from the boundary when
    # (4/h^2)[sin^2(kappa h cos t / 2) + sin^2(kappa h sin t / 2)] = k^2.
    nx, ny = 20, 16
    c = 1.7 * C_REF
    P = homogeneous_problem(nx, ny, c=c)
    h = P.h
    k2 = (C_REF / c) ** 2
    f = lambda kap: 4 / h ** 2 * (math.sin(kap * h * math.cos(theta) / 2) ** 2
                                  + math.sin(kap * h * math.sin(theta) / 2) ** 2) - k2
    kappa = optimize.brentq(f, 1e-6, math.pi / h * 0.99)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    u = np.exp(1j * kappa * (x[None, :] * math.cos(theta) + y[:, None] * math.sin(theta)))
    Au = hz.op_apply(P, u)
    scale = 8.0 / h ** 2 + k2
    assert np.max(np.abs(Au[1:-1, 1:-1])) <= 1e-12 * scale
    # the boundary rows are not annihilated (the outside values are zero, not the wave)
    assert np.max(np.abs(Au[0, :])) > 1e-3 * scale


def test_dense_assembly_matches_apply():
    s = c1_system(0)
    # shrink to a tiny grid with a PML, keeping a heterogeneous velocity
    c = s.c[30:52, 28:46]
    P = hz.Problem(c, 4, H_10PPW, 1.0, 2.0, C_REF)
    A = hz.assemble_dense(P)
    rng = np.random.default_rng(0)
    for _ in range(3):
        u = rng.standard_normal(P.n) + 1j * rng.standard_normal(P.n)
        y1 = hz.op_apply(P, u.reshape(P.ny, P.nx)).ravel()
        y2 = A @ u
        assert np.linalg.norm(y1 - y2) <= 1e-14 * np.linalg.norm(y2)
        w = rng.standard_normal(P.n) + 1j * rng.standard_normal(P.n)
        a1 = hz.op_adjoint(P, w.reshape(P.ny, P.nx)).ravel()
        a2 = A.conj().T @ w
        assert np.linalg.norm(a1 - a2) <= 1e-14 * np.linalg.norm(a2)


def test_adjoint_dot_test():
    s = c1_system(1)
    P = hz.Problem(s.c, s.npml, H_10PPW, 1.0, 2.0, C_REF)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((P.ny, P.nx)) + 1j * rng.standard_normal((P.ny, P.nx))
    w = rng.standard_normal((P.ny, P.nx)) + 1j * rng.standard_normal((P.ny, P.nx))
    lhs = np.vdot(w, hz.op_apply(P, u))        # <Au, w> = w^H A u
    rhs = np.vdot(hz.op_adjoint(P, w), u)      # <u, A^H w> = (A^H w)^H u
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs) * 10


def test_pml_profile_and_symmetry():
    # sigma is zero on the inner nodes, sigma_max at the outermost node, quadratic in between,
    # and the coefficients are mirror-symmetric: a+[i] == a-[n-1-i].
    n, p = 30, 6
    s = np.arange(n)
    sig = hz.pml_sigma(s, n, p, 2.0)
    assert np.all(sig[p:n - p] == 0)
    assert sig[0] == pytest.approx(2.0) and sig[-1] == pytest.approx(2.0)
    assert sig[p // 2] == pytest.approx(2.0 * 0.25)
    ap, am = hz.axis_coefficients(n, p, 0.5, 1.0, 2.0)
    assert np.allclose(ap, am[::-1], rtol=0, atol=1e-15 * abs(ap).max())
    assert np.allclose(ap[p:n - p - 1], 1 / 0.25)
    assert np.all(ap[:p].imag < 0)       # 1 / (gamma gamma) with gamma = 1 + i sigma has Im < 0


def test_free_space_green_function_with_pml():
    # A point source f = delta / h^2 in a homogeneous medium radiates -(i/4) H0^(1)(k r) (outgoing
    # waves under the radiation condition of eq. (1)). With the PML absorbing the outgoing wave, the
    # discrete solution matches it to a few per cent a few wavelengths from the source; a PML with the
    # wrong stretch sign or without damping reflects and fails this by a wide margin.
    nint, p = 44, 12
    nt = nint + 2 * p
    P = homogeneous_problem(nt, nt, npml=p, sigma_max=2.0, h=2 * math.pi / 12)
    A = hz.assemble_dense(P)
    b = np.zeros((nt, nt), np.complex128)
    ci = nt // 2
    b[ci, ci] = 1.0 / P.h ** 2
    u = np.linalg.solve(A, b.ravel()).reshape(nt, nt)
    jj, ii = np.meshgrid(np.arange(nt), np.arange(nt), indexing="ij")
    r = np.hypot(ii - ci, jj - ci) * P.h
    ring = (r > 3 * P.h) & (r < (nint / 2 - 2) * P.h)
    g = -0.25j * special.hankel1(0, r[ring])
    err = np.linalg.norm(u[ring] - g) / np.linalg.norm(g)
    assert err < 0.08, err
    # the field decays through the layer
    assert np.abs(u[0, :]).max() < 0.05 * np.abs(u[p, p:-p]).max()
    # the opposite stretch sign reflects strongly
    bad = hz.Problem(P.c, p, P.h, 1.0, -2.0, C_REF)
    ub = np.linalg.solve(hz.assemble_dense(bad), b.ravel()).reshape(nt, nt)
    errb = np.linalg.norm(ub[ring] - g) / np.linalg.norm(g)
    assert errb > 3 * err


def test_wavenumber_units():
    # k = omega / c~ with c~ = c / c_ref: the 1500 m/s background has k = 1 and 10 nodes per
    # wavelength at h = 2 pi / 10
    P = homogeneous_problem(4, 4)
    assert np.allclose(P.k2, 1.0)
    assert 2 * math.pi / math.sqrt(P.k2[0, 0]) / P.h == pytest.approx(10.0)
