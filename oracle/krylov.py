"""GMRES solvers for the preconditioned system (oracle, complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.3 solves the preconditioned system M_alpha A u = M_alpha f with GMRES
(Saad & Schultz).  The paper does not state restart, initial guess or which
residual its tolerance refers to.  Readings used here:

* ``fgmres``: right-preconditioned flexible GMRES(k) -- A M y = f, u = M y,
  storing the preconditioned directions Z so that an inexact (e.g. single
  precision) preconditioner is allowed; x0 = 0 unless given; stop when the
  true residual ||f - A u||_2 / ||f||_2 <= tol (checked with the Arnoldi
  estimate inside a cycle, confirmed with an explicit residual at the end of
  every cycle).  Modified Gram-Schmidt, complex Givens rotations.
* ``gmres_left``: the paper's left-preconditioned form, stopping on the
  preconditioned residual ||M(f - A u)|| / ||M f||; used only to compare
  iteration counts with the paper's tables.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: List[float] = field(default_factory=list)   # Arnoldi residual estimates / ||f||
    true_history: List[float] = field(default_factory=list)  # explicit residuals at cycle ends


def _givens(a: complex, b: complex):
    """Complex rotation G = [[c, s], [-conj(s), c]] with G (a, b)^t = (r, 0)^t, c real."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def fgmres(matvec: Callable, precond: Callable, f: np.ndarray, restart: int = 20,
           tol: float = 1e-6, maxit: int = 1000, x0: Optional[np.ndarray] = None) -> KrylovResult:
    f = np.asarray(f, dtype=np.complex128)
    N = f.shape[0]
    fnorm = np.linalg.norm(f)
    x = np.zeros(N, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if fnorm == 0.0:
        return KrylovResult(np.zeros(N, dtype=np.complex128), 0, 0.0, True)
    r = f - matvec(x)
    beta = np.linalg.norm(r)
    res = KrylovResult(x, 0, beta / fnorm, beta / fnorm <= tol)
    res.true_history.append(beta / fnorm)
    if res.converged:
        return res
    total = 0
    while True:
        k = restart
        V = np.zeros((k + 1, N), dtype=np.complex128)
        Z = np.zeros((k, N), dtype=np.complex128)
        H = np.zeros((k + 1, k), dtype=np.complex128)
        cs = np.zeros(k)
        sn = np.zeros(k, dtype=np.complex128)
        g = np.zeros(k + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(k):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                           # previous rotations
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            est = abs(g[j + 1]) / fnorm
            res.history.append(est)
            if est <= tol or total >= maxit or H[j, j] == 0:
                break
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):              # back substitution, H upper triangular
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        x = x + Z[:j_done].T @ y
        r = f - matvec(x)
        beta = np.linalg.norm(r)
        rel = beta / fnorm
        res.true_history.append(rel)
        res.x, res.iters, res.relres = x, total, rel
        if rel <= tol:
            res.converged = True
            return res
        if total >= maxit:
            res.converged = False
            return res


def gmres_left(matvec: Callable, precond: Callable, f: np.ndarray, tol: float = 1e-3,
               maxit: int = 500) -> KrylovResult:
    """Unrestarted GMRES on M A u = M f (left preconditioning, the paper's formulation)."""
    f = np.asarray(f, dtype=np.complex128)
    N = f.shape[0]
    b = precond(f)
    bnorm = np.linalg.norm(b)
    V = [b / bnorm]
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = bnorm
    hist = []
    j_done = 0
    for j in range(maxit):
        w = precond(matvec(V[j]))
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
        for i in range(j):
            hi, hi1 = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * hi + sn[i] * hi1
            H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        j_done = j + 1
        hist.append(abs(g[j + 1]) / bnorm)
        if hist[-1] <= tol:
            break
    y = np.zeros(j_done, dtype=np.complex128)
    for i in range(j_done - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
    x = np.stack(V[:j_done], axis=1) @ y
    r = f - matvec(x)
    return KrylovResult(x, j_done, np.linalg.norm(r) / np.linalg.norm(f), hist[-1] <= tol, hist)
