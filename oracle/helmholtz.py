"""Oracle: the discrete 2-D Helmholtz operator with a perfectly matched layer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.1: eq. (1) (Laplacian + k^2 with the Sommerfeld condition,
k = omega / c), eq. (2) (quadratic PML damping, zero in the inner domain) and
eq. (3) (A(c) = Laplacian + k^2 acting on grid vectors). The paper
differentiates spectrally; this oracle uses the second-order five-point
finite-difference form of the stretched Laplacian (the reading adopted for the
build), with homogeneous Dirichlet values outside the grid.

Grid: nodes i = 0..nx_t-1 along x and j = 0..ny_t-1 along y, where the totals
include npml PML cells on each side; a grid vector u has shape [ny_t, nx_t]
(flattened index j * nx_t + i). Position s along an axis (a node or a
half-node) lies d(s) = max(0, npml - s, s - (n_t - 1 - npml)) cells deep in
the layer, has damping sigma(s) = sigma_max (d / npml)^2 and stretch
gamma(s) = 1 + i sigma(s) / omega (complex coordinate stretching; the sign
selects the outgoing wave exp(+i k r) fixed by the radiation condition).

The stretched second derivative at node i is
  a_plus[i] (u[i+1] - u[i]) - a_minus[i] (u[i] - u[i-1]),
  a_plus[i]  = 1 / (h^2 gamma(i) gamma(i + 1/2)),
  a_minus[i] = 1 / (h^2 gamma(i) gamma(i - 1/2)).
"""
from __future__ import annotations

import numpy as np


def pml_depth(s, n_total: int, npml: int):
    """Depth (in cells) of position s into the layer; 0 in the inner domain."""
    s = np.asarray(s, dtype=np.float64)
    return np.maximum(0.0, np.maximum(npml - s, s - (n_total - 1 - npml)))


def pml_sigma(s, n_total: int, npml: int, sigma_max: float):
    """Eq. (2): sigma_max * (depth / layer width)^2 inside the layer, 0 elsewhere."""
    if npml == 0:
        return np.zeros_like(np.asarray(s, dtype=np.float64))
    d = pml_depth(s, n_total, npml)
    return sigma_max * (d / npml) ** 2


def axis_coefficients(n_total: int, npml: int, h: float, omega: float, sigma_max: float):
    """(a_plus, a_minus), complex128 [n_total], for one axis."""
    i = np.arange(n_total, dtype=np.float64)
    g = lambda s: 1.0 + 1j * pml_sigma(s, n_total, npml, sigma_max) / omega
    a_plus = 1.0 / (h * h * g(i) * g(i + 0.5))
    a_minus = 1.0 / (h * h * g(i) * g(i - 0.5))
    return a_plus, a_minus


def wavenumber_sq(c, omega: float, c_ref: float):
    """k^2 = (omega / c~)^2 with the nondimensional velocity c~ = c / c_ref."""
    c = np.asarray(c, dtype=np.float64)
    return (omega * c_ref / c) ** 2


class Problem:
    """One discrete Helmholtz system: grid, PML coefficients and k^2 (all FP64)."""

    def __init__(self, c, npml: int, h: float, omega: float = 1.0, sigma_max: float = 2.0,
                 c_ref: float = 1500.0):
        c = np.asarray(c, dtype=np.float64)
        self.ny, self.nx = c.shape
        self.npml, self.h, self.omega, self.sigma_max, self.c_ref = npml, h, omega, sigma_max, c_ref
        self.c = c
        self.k2 = wavenumber_sq(c, omega, c_ref)
        self.axp, self.axm = axis_coefficients(self.nx, npml, h, omega, sigma_max)
        self.ayp, self.aym = axis_coefficients(self.ny, npml, h, omega, sigma_max)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def sigma_nodes(self):
        """(sigma_x, sigma_y) at the nodes, each [ny, nx] float64."""
        sx = pml_sigma(np.arange(self.nx), self.nx, self.npml, self.sigma_max)
        sy = pml_sigma(np.arange(self.ny), self.ny, self.npml, self.sigma_max)
        return np.broadcast_to(sx[None, :], (self.ny, self.nx)).copy(), \
            np.broadcast_to(sy[:, None], (self.ny, self.nx)).copy()


def _shift(u, dj: int, di: int):
    """out[j, i] = u[j + dj, i + di], zero outside the grid."""
    out = np.zeros_like(u)
    ny, nx = u.shape
    js = slice(max(0, -dj), min(ny, ny - dj))
    is_ = slice(max(0, -di), min(nx, nx - di))
    jt = slice(max(0, dj), min(ny, ny + dj))
    it = slice(max(0, di), min(nx, nx + di))
    out[js, is_] = u[jt, it]
    return out


def op_apply(p: Problem, u):
    """(A u)[j,i] = a+x[i](u[i+1]-u[i]) - a-x[i](u[i]-u[i-1]) + (same along y) + k^2 u."""
    u = np.asarray(u, dtype=np.complex128).reshape(p.ny, p.nx)
    axp, axm = p.axp[None, :], p.axm[None, :]
    ayp, aym = p.ayp[:, None], p.aym[:, None]
    return (axp * (_shift(u, 0, 1) - u) - axm * (u - _shift(u, 0, -1))
            + ayp * (_shift(u, 1, 0) - u) - aym * (u - _shift(u, -1, 0))
            + p.k2 * u)


def op_diagonal(p: Problem):
    """Diagonal entries of A: k^2 - a+x - a-x - a+y - a-y, [ny, nx]."""
    return p.k2 - p.axp[None, :] - p.axm[None, :] - p.ayp[:, None] - p.aym[:, None]


def op_adjoint(p: Problem, w):
    """(A^H w)[j,i] = conj(a-x[i+1]) w[i+1] + conj(a+x[i-1]) w[i-1] + (y alike) + conj(diag) w.

    Row (j,i) of A couples to (j,i+1) with a+x[i] and to (j,i-1) with a-x[i]; A^H takes the
    conjugate transpose, so node i collects a-x[i+1] from its right neighbour and a+x[i-1] from
    its left neighbour. Terms that would reference nodes outside the grid are dropped.
    """
    w = np.asarray(w, dtype=np.complex128).reshape(p.ny, p.nx)
    cxm_r = np.zeros(p.nx, np.complex128)   # conj(a-x[i+1]) for i < nx-1
    cxm_r[:-1] = np.conj(p.axm[1:])
    cxp_l = np.zeros(p.nx, np.complex128)   # conj(a+x[i-1]) for i > 0
    cxp_l[1:] = np.conj(p.axp[:-1])
    cym_r = np.zeros(p.ny, np.complex128)
    cym_r[:-1] = np.conj(p.aym[1:])
    cyp_l = np.zeros(p.ny, np.complex128)
    cyp_l[1:] = np.conj(p.ayp[:-1])
    return (cxm_r[None, :] * _shift(w, 0, 1) + cxp_l[None, :] * _shift(w, 0, -1)
            + cym_r[:, None] * _shift(w, 1, 0) + cyp_l[:, None] * _shift(w, -1, 0)
            + np.conj(op_diagonal(p)) * w)


def assemble_dense(p: Problem):
    """The n x n matrix entry by entry from the stencil formula (only for small grids)."""
    n = p.n
    if n > 10000:
        raise ValueError("dense assembly is for tiny grids only")
    A = np.zeros((n, n), np.complex128)
    for j in range(p.ny):
        for i in range(p.nx):
            r = j * p.nx + i
            A[r, r] = p.k2[j, i] - p.axp[i] - p.axm[i] - p.ayp[j] - p.aym[j]
            if i + 1 < p.nx:
                A[r, r + 1] = p.axp[i]
            if i - 1 >= 0:
                A[r, r - 1] = p.axm[i]
            if j + 1 < p.ny:
                A[r, r + p.nx] = p.ayp[j]
            if j - 1 >= 0:
                A[r, r - p.nx] = p.aym[j]
    return A
