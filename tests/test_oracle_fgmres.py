"""Pins of the oracle's FGMRES against dense LU, brute-force Krylov least squares and exact
invariants (Algorithm 1, eq. (4), eq. (13))."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fgmres as fg
from oracle import helmholtz as hz
from oracle import unet
from synth import C_REF, H_10PPW, he_uniform, rng_for, skull_ring_velocity, gaussian_sources


def tiny_problem(seed=0, nx=10, p=4):
    nt = nx + 2 * p
    c = skull_ring_velocity(nt, p, rng_for(7, 0, seed), rings=1, thickness=2.0)
    P = hz.Problem(c, p, H_10PPW, 1.0, 2.0, C_REF)
    b = gaussian_sources(nt, p, rng_for(7, 1, seed), nsrc=2) if nx >= 10 else \
        np.random.default_rng(seed).standard_normal((nt, nt)) + 0j
    return P, b


def ops(P):
    A = lambda x: hz.op_apply(P, x.reshape(P.ny, P.nx)).ravel()
    return A


def test_givens_rotation():
    for a, b in [(1 + 2j, 0.5), (0j, 3.0), (-2 + 0.1j, 4.0), (1e-300 + 0j, 1.0)]:
        c, s, r = fg.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) <= 1e-15 * abs(r) and abs(out[0] - r) <= 1e-15 * abs(r)
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-15)


def test_full_gmres_matches_dense_lu_and_terminates():
    P, b = tiny_problem(0, nx=10, p=4)            # n = 324
    A = hz.assemble_dense(P)
    x_lu = np.linalg.solve(A, b.ravel())
    r = fg.fgmres(ops(P), lambda v: v, b, m=P.n, tol=1e-12, maxit=P.n)
    assert r.status == fg.CONVERGED
    assert r.its <= P.n
    assert np.linalg.norm(r.x - x_lu) <= 1e-8 * np.linalg.norm(x_lu)
    assert np.linalg.norm(A @ r.x - b.ravel()) / np.linalg.norm(b) <= 1e-12


def test_exact_termination_in_n_steps():
    # full GMRES on an n x n system reaches the exact solution within n steps
    P, _ = tiny_problem(1, nx=2, p=2)           # n = 36
    b = np.random.default_rng(3).standard_normal(P.n) + 1j * np.random.default_rng(4).standard_normal(P.n)
    r = fg.fgmres(ops(P), lambda v: v, b, m=P.n, tol=1e-13, maxit=P.n)
    assert r.status == fg.CONVERGED and r.its <= P.n


def test_arnoldi_relation_orthogonality_and_monotone_residual():
    P, b = tiny_problem(2, nx=12, p=4)
    specs = unet.layer_specs(2, 4, 5)
    theta = he_uniform(unet.init_shapes(specs), np.random.default_rng(5)).astype(np.float64)
    M = lambda v: unet.precond_apply(theta, specs, P, v.reshape(P.ny, P.nx)).ravel()
    A = ops(P)
    m = 25
    r = fg.fgmres(A, M, b, m=m, tol=1e-14, maxit=m, keep_basis=True)
    cyc = r.last_cycle
    V, Z, H, k = cyc["V"], cyc["Z"], cyc["H"], cyc["k"]
    AZ = np.stack([A(z) for z in Z], axis=1)
    VH = V.T @ H
    assert np.linalg.norm(AZ - VH) <= 1e-13 * np.linalg.norm(AZ)          # eq. (4)
    assert np.max(np.abs(V.conj() @ V.T - np.eye(V.shape[0]))) <= 1e-12   # V^H V = I
    est = np.array(r.est_history)
    assert np.all(np.diff(est) <= 0)                                       # |g_{j+1}| = |s_j| |g_j|
    # the Givens estimate equals the true residual of the cycle's iterate
    true = np.linalg.norm(b.ravel() - A(r.x)) / np.linalg.norm(b)
    assert abs(true - est[-1]) <= 1e-10 * max(true, 1e-300) + 1e-13


def test_fixed_linear_preconditioner_is_gmres_on_AM():
    # with z = M v for a fixed matrix M, step k minimises ||b - A M t|| over the Krylov space
    # K_k(AM, b): compare the running residual with a brute-force least squares on an
    # orthonormalised Krylov basis
    P, b = tiny_problem(3, nx=10, p=4)
    A = hz.assemble_dense(P)
    rng = np.random.default_rng(6)
    Mmat = np.eye(P.n) + 0.05 * (rng.standard_normal((P.n, P.n)) + 1j * rng.standard_normal((P.n, P.n))) / np.sqrt(P.n)
    bb = b.ravel()
    r = fg.fgmres(lambda x: A @ x, lambda v: Mmat @ v, bb, m=12, tol=1e-30, maxit=12)
    AM = A @ Mmat
    K = [bb / np.linalg.norm(bb)]
    for k in range(1, 13):
        Q, _ = np.linalg.qr(np.stack(K, axis=1))
        Y = AM @ Q
        t, *_ = np.linalg.lstsq(Y, bb, rcond=None)
        brute = np.linalg.norm(bb - Y @ t) / np.linalg.norm(bb)
        assert abs(brute - r.est_history[k - 1]) <= 1e-8 * brute
        K.append(AM @ K[-1])
        K[-1] /= np.linalg.norm(K[-1])


def test_restarted_matches_scipy_solution_and_true_residual_monotone():
    P, b = tiny_problem(4, nx=10, p=4)
    A = hz.assemble_dense(P)
    r = fg.fgmres(lambda x: A @ x, lambda v: v, b, m=15, tol=1e-10, maxit=4000)
    assert r.status == fg.CONVERGED
    th = np.array(r.true_history)
    assert np.all(np.diff(th) <= 1e-12)     # restarted GMRES never increases the residual
    xs, info = spla.gmres(A, b.ravel(), rtol=1e-12, restart=15, maxiter=4000)
    assert info == 0
    assert np.linalg.norm(r.x - xs) <= 1e-7 * np.linalg.norm(xs)


def test_degenerate_cases():
    P, b = tiny_problem(5, nx=10, p=4)
    A = ops(P)
    # zero right-hand side: x = 0, converged, no iterations
    r = fg.fgmres(A, lambda v: v, np.zeros(P.n), m=5, tol=1e-6, maxit=10)
    assert r.status == fg.CONVERGED and r.its == 0 and not np.any(r.x)
    # exact initial guess: converged at once
    x_lu = np.linalg.solve(hz.assemble_dense(P), b.ravel())
    r = fg.fgmres(A, lambda v: v, b, m=5, tol=1e-10, maxit=10, x0=x_lu)
    assert r.status == fg.CONVERGED and r.its == 0
    # zero preconditioner: Z is rank deficient -> breakdown
    r = fg.fgmres(A, lambda v: 0 * v, b, m=5, tol=1e-6, maxit=10)
    assert r.status == fg.BREAKDOWN and r.its == 1
    # iteration cap
    r = fg.fgmres(A, lambda v: v, b, m=5, tol=1e-14, maxit=7)
    assert r.status == fg.NOT_CONVERGED and r.its == 7 and r.cycles == 2
