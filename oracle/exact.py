"""Exact dense sweeping factorisation (oracle, complex128, small n only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.1, eq. Afact: block LDL^t of the block-tridiagonal A layer by layer,
S_1 = A_11, S_m = A_mm - A_{m,m-1} S_{m-1}^{-1} A_{m-1,m}, with T_m = S_m^{-1}
(Algorithm 1), and u = A^{-1} f by forward substitution, diagonal solves and
backward substitution (Algorithm 2).  O(n^4) setup: used only as a pin for
n <= ~40.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _blocks(A: sp.spmatrix, n: int):
    A = A.tocsr()
    def blk(a: int, b: int) -> np.ndarray:   # 1-based layer indices
        return A[(a - 1) * n:a * n, (b - 1) * n:b * n].toarray()
    return blk


def setup_exact(A: sp.spmatrix, n: int):
    """Algorithm 1: T_m = S_m^{-1}, m = 1..n (dense n x n each)."""
    blk = _blocks(A, n)
    T = [None] * (n + 1)
    S = blk(1, 1)
    T[1] = np.linalg.inv(S)
    for m in range(2, n + 1):
        S = blk(m, m) - blk(m, m - 1) @ T[m - 1] @ blk(m - 1, m)
        T[m] = np.linalg.inv(S)
    return T


def solve_exact(A: sp.spmatrix, n: int, T, f: np.ndarray) -> np.ndarray:
    """Algorithm 2: u = A^{-1} f from the exact sweeping factorisation."""
    blk = _blocks(A, n)
    u = [None] + [np.array(f[(m - 1) * n:m * n], dtype=np.complex128) for m in range(1, n + 1)]
    for m in range(1, n):
        u[m + 1] = u[m + 1] - blk(m + 1, m) @ (T[m] @ u[m])
    for m in range(1, n + 1):
        u[m] = T[m] @ u[m]
    for m in range(n - 1, 0, -1):
        u[m] = u[m] - T[m] @ (blk(m, m + 1) @ u[m + 1])
    return np.concatenate(u[1:])
