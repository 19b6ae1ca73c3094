"""Oracle: restarted flexible GMRES with a (possibly nonlinear) right preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Algorithm 1 and eq. (4) of Section 2.2 (generalized Arnoldi relation
A Z_k = V_{k+1} Hbar_k with z_i = M_i(v_i)), the stopping rule eq. (13) and the
cycle/iteration bookkeeping of Section 4. Readings adopted where the paper is
silent: h_ij = v_i^H w; x0 = 0 unless given; m is the cycle length and
``maxit`` caps the total number of preconditioner applications; the least
squares problem is solved by complex Givens rotations whose running residual
|g_{j+1}| ends a cycle early once |g_{j+1}| / ||b|| <= tol, and a solve counts
as converged only when the true residual ||b - A x|| / ||b|| recomputed at the
end of a cycle is <= tol.

Givens convention: for the pair (a, b) = (h_jj, h_{j+1,j}) with rho =
sqrt(|a|^2 + |b|^2), c = |a| / rho (real) and s = (a / |a|) conj(b) / rho
(s = 1 when a = 0); the rotation maps (x, y) to (c x + s y, -conj(s) x + c y).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, -4


@dataclass
class Result:
    x: np.ndarray
    status: int
    its: int
    cycles: int
    est_history: list = field(default_factory=list)    # |g_{j+1}| / ||b|| after every step
    true_history: list = field(default_factory=list)   # ||b - A x|| / ||b|| at every cycle start and end
    true_relres: float = np.nan
    last_cycle: dict = field(default_factory=dict)     # V, Z, H of the final cycle (for invariants)


def givens(a: complex, b: complex):
    """(c, s, r): c real, s complex with [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    rho = np.hypot(abs(a), abs(b))
    if rho == 0.0:
        return 1.0, 0.0 + 0.0j, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b) + 0.0j
    ph = a / abs(a)
    c = abs(a) / rho
    s = ph * np.conj(b) / rho
    return c, s, ph * rho


def fgmres(apply_A, apply_M, b, *, m: int, tol: float, maxit: int, x0=None,
           breakdown_tol: float = 1e-14, keep_basis: bool = False) -> Result:
    """Restarted FGMRES(m) on A x = b; apply_M(v) is the (flexible) preconditioner.

    All vectors are complex128 1-D arrays. Returns a Result (see its fields).
    """
    b = np.asarray(b, dtype=np.complex128).ravel()
    n = b.size
    x = np.zeros(n, np.complex128) if x0 is None else np.asarray(x0, np.complex128).ravel().copy()
    nb = np.linalg.norm(b)
    res = Result(x=x, status=NOT_CONVERGED, its=0, cycles=0)
    if nb == 0.0:
        res.x[:] = 0.0
        res.status, res.true_relres = CONVERGED, 0.0
        return res
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        rel = beta / nb
        res.true_history.append(rel)
        res.true_relres = rel
        if rel <= tol:
            res.status = CONVERGED
            break
        if res.its >= maxit:
            res.status = NOT_CONVERGED
            break
        if not np.isfinite(beta):
            res.status = BREAKDOWN
            break
        res.cycles += 1
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), np.complex128)
        R = np.zeros((m + 1, m), np.complex128)
        cs, sn = np.zeros(m), np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        k = 0            # number of columns completed in this cycle
        broke = False
        for j in range(m):
            z = apply_M(V[j])
            Z.append(z)
            w = apply_A(z)
            wnorm0 = np.linalg.norm(w)
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            col = H[:j + 2, j].copy()
            for i in range(j):              # previous rotations
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
                col[i] = t
            c_, s_, rr = givens(col[j], col[j + 1])
            cs[j], sn[j] = c_, s_
            col[j], col[j + 1] = rr, 0.0
            R[:j + 2, j] = col
            g[j + 1] = -np.conj(s_) * g[j]
            g[j] = c_ * g[j]
            res.its += 1
            k = j + 1
            est = abs(g[j + 1]) / nb
            res.est_history.append(est)
            if hnext <= breakdown_tol * wnorm0:
                broke = True
                break
            V.append(w / hnext)
            if est <= tol or res.its >= maxit:
                break
        while k > 0 and R[k - 1, k - 1] == 0:   # a zero pivot: z_k added nothing (rank-deficient Z)
            k -= 1
        y = back_substitute(R[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        res.x = x
        if keep_basis:
            res.last_cycle = dict(V=np.array(V), Z=np.array(Z), H=H[:k + 1, :k].copy(), k=k, g=g[:k + 1].copy())
        if broke:
            r = b - apply_A(x)
            rel = np.linalg.norm(r) / nb
            res.true_history.append(rel)
            res.true_relres = rel
            res.status = CONVERGED if rel <= tol else BREAKDOWN
            break
    res.x = x
    return res


def back_substitute(R, g):
    """Solve the upper triangular system R y = g by back substitution (written out)."""
    k = R.shape[0]
    y = np.zeros(k, np.complex128)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
    return y
