"""Discrete PML-stretched Helmholtz operator (oracle, complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2.1 of Engquist & Ying, "Sweeping preconditioner for the
Helmholtz equation: moving perfectly matched layers" (2010):

* the quadratic damping profile sigma (eq. sigma) and the stretch
  s = (1 + i sigma / omega)^{-1};
* the symmetric form  d1 (s1/s2 d1) + d2 (s2/s1 d2) + omega^2 / (s1 s2 c^2);
* its 5-point discretisation (eq. helmd) on the interior grid with spacing
  h = 1/(n+1) and zero Dirichlet values outside, rows ordered row by row;
* the modified operator A_alpha with omega^2 -> (omega + i alpha)^2
  (eq. helmalpha, Section 2.3).

Readings of points the paper leaves open (each one also listed in the design notes):

* PML constant C: the paper only asks for a positive constant independent of
  omega; ``Params.C`` defaults to 20.
* Width: a width ``w`` means ``w`` damped grid rows, eta = (w+1) h, so the
  damped strip plus the first undamped row spans B = w+1 rows (the moving-PML
  subproblem of Section 2.2 has B rows).  ``b_convention=1`` switches to the
  literal eta = w h, B = w.
* The shift alpha enters only the mass term; s keeps the real omega.
* PML on all four sides (Section 3.1): sigma is two-sided in x1 and in x2.
* The "sum of the four coefficients" on the diagonal of eq. helmd includes
  the half-point coefficients that reach a Dirichlet boundary.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Params:
    n: int                 # interior points per side
    omega: float           # angular frequency
    alpha: float = 2.0     # shift of the preconditioner's operator
    pml_w: int = 12        # physical PML: damped rows per side
    mpml_w: int = 12       # moving PML: damped rows
    C: float = 20.0        # PML strength constant
    b_convention: int = 0  # 0: eta=(w+1)h, B=w+1 ; 1: eta=wh, B=w

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def B(self) -> int:
        """Rows of a moving-PML subproblem (block size of the x2-first ordering)."""
        return self.mpml_w + 1 if self.b_convention == 0 else self.mpml_w

    @property
    def eta_phys(self) -> float:
        w = self.pml_w + 1 if self.b_convention == 0 else self.pml_w
        return w * self.h

    @property
    def eta_move(self) -> float:
        return self.B * self.h

    @property
    def mid(self) -> int:
        """Middle layer of the two-front sweep: (n+1)/2 for odd n, n/2+1 for even n."""
        return (self.n + 1) // 2 if self.n % 2 == 1 else self.n // 2 + 1


def sigma_low(t, eta: float, C: float):
    """Damping profile of a layer occupying [0, eta): (C/eta)((t-eta)/eta)^2, zero beyond (eq. sigma)."""
    t = np.asarray(t, dtype=np.float64)
    out = (C / eta) * ((t - eta) / eta) ** 2
    return np.where((t >= 0.0) & (t < eta), out, 0.0)


def sigma_phys(t, eta: float, C: float):
    """Two-sided profile of the unit interval: damping near t=0 and near t=1 (eq. sigma, sigma_1)."""
    t = np.asarray(t, dtype=np.float64)
    return sigma_low(t, eta, C) + sigma_low(1.0 - t, eta, C)


def stretch(sigma, omega: float):
    """s = (1 + i sigma/omega)^{-1} (Section 2.1)."""
    return 1.0 / (1.0 + 1j * np.asarray(sigma, dtype=np.float64) / omega)


def strip_operator(c_rows: np.ndarray, h: float, s1_node: np.ndarray, s1_half: np.ndarray,
                   s2_node: np.ndarray, s2_half: np.ndarray, kappa: complex) -> sp.csr_matrix:
    """5-point operator of eq. helmd on a horizontal strip of ``R`` grid rows.

    c_rows   (R, n)   velocity on the strip's rows (row-major: [local row, i])
    s1_node  (n,)     s1 at x1 = ih, i = 1..n
    s1_half  (n+1,)   s1 at x1 = (i+1/2)h, i = 0..n
    s2_node  (R,)     s2 at the strip's rows
    s2_half  (R+1,)   s2 at the half rows below the first row, between rows, above the last
    kappa             omega (operator A) or omega + i alpha (A_alpha)

    Unknowns are ordered row by row: index r*n + (i-1) for local row r (0-based).
    Neighbours outside the strip are zero (Dirichlet); the diagonal still sums
    all four half-point coefficients.
    """
    R, n = c_rows.shape
    inv_h2 = 1.0 / (h * h)
    # ax[r, k] couples (k, r) and (k+1, r): (s1/s2) at ((k+1/2)h, row r), k = 0..n
    ax = (s1_half[None, :] / s2_node[:, None]) * inv_h2            # (R, n+1)
    # ay[k, i] couples rows k-1 and k at column i: (s2/s1) at (ih, half row k), k = 0..R
    ay = (s2_half[:, None] / s1_node[None, :]) * inv_h2             # (R+1, n)
    mass = kappa ** 2 / (s1_node[None, :] * s2_node[:, None] * c_rows ** 2)
    diag = mass - (ax[:, :-1] + ax[:, 1:] + ay[:-1, :] + ay[1:, :])

    idx = np.arange(R * n).reshape(R, n)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # x1 neighbours inside the strip: (i, r) -- (i+1, r), coefficient ax[r, i] (half point i+1/2)
    a = ax[:, 1:-1]
    rows += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals += [a.ravel(), a.ravel()]
    # x2 neighbours: (i, r) -- (i, r+1), coefficient ay[r+1, i]
    b = ay[1:-1, :]
    rows += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals += [b.ravel(), b.ravel()]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(R * n, R * n)).tocsr()
    A.sum_duplicates()
    return A


def x1_profiles(p: Params):
    """s1 at the nodes ih (i=1..n) and half points (i+1/2)h (i=0..n), physical two-sided profile."""
    h = p.h
    t_node = h * np.arange(1, p.n + 1)
    t_half = h * (np.arange(0, p.n + 1) + 0.5)
    s_node = stretch(sigma_phys(t_node, p.eta_phys, p.C), p.omega)
    s_half = stretch(sigma_phys(t_half, p.eta_phys, p.C), p.omega)
    return s_node, s_half


def x2_phys_profiles(p: Params, rows: np.ndarray):
    """Physical s2 at the given 1-based rows and at their half rows (below each row and above the last).

    ``rows`` must be consecutive and increasing.
    """
    h = p.h
    rows = np.asarray(rows)
    t_node = h * rows
    t_half = h * (np.arange(rows[0] - 1, rows[-1] + 1) + 0.5)
    return (stretch(sigma_phys(t_node, p.eta_phys, p.C), p.omega),
            stretch(sigma_phys(t_half, p.eta_phys, p.C), p.omega))


def assemble(p: Params, c: np.ndarray, shifted: bool = False) -> sp.csr_matrix:
    """A (shifted=False, kappa=omega) or A_alpha (shifted=True, kappa=omega+i alpha) on the whole grid.

    eq. helmd with the PML of eq. sigma on all four sides; eq. helmalpha for the shift.
    """
    n = p.n
    c2 = np.asarray(c, dtype=np.float64).reshape(n, n)
    s1n, s1h = x1_profiles(p)
    s2n, s2h = x2_phys_profiles(p, np.arange(1, n + 1))
    kappa = p.omega + 1j * p.alpha if shifted else p.omega + 0j
    return strip_operator(c2, p.h, s1n, s1h, s2n, s2h, kappa)


def row_coupling(p: Params, j: int) -> np.ndarray:
    """Entries of the diagonal block A_{j+1,j} = A_{j,j+1}: (s2/s1)/h^2 at (ih, (j+1/2)h), i=1..n."""
    s1n, _ = x1_profiles(p)
    s2 = stretch(sigma_phys(p.h * (j + 0.5), p.eta_phys, p.C), p.omega)
    return s2 / s1n / (p.h * p.h)
