"""Moving-PML subproblems and the approximate sweeping LDL^t (oracle, complex128).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.2 (moving PML): the Schur inverse T_m of layer m is replaced by
T~_m, defined through the operator H_m of eq. helma discretised on the strip
of B rows ending at layer m, whose x2-profile is the PML pushed right next to
the layer: s2^m(x2) = s(sigma_2(x2 - (m-B)h)).  T~_m g is the last-row block of
H_m^{-1} (0, ..., 0, g).  H_m is factored after the permutation P_m to the
x2-first ordering, in which it is banded; here with LAPACK's partial-pivoting
band LU (zgbtrf / zgbtrs), a different route from the GPU's block recurrence.

Section 2.3: Algorithm 3 (setup) factors the front F (the first B layers,
H_F = A_{F,F}) and every moving-PML subproblem; Algorithm 4 (application)
runs the forward substitution, the diagonal T~ applications and the backward
substitution.  With PML on all sides the sweep runs two fronts, upward from
x2 = 0 (F, B+1, ..., c-1) and downward from x2 = 1 (E, n-B, ..., c+1), and
ends at the middle layer c with moving PMLs on both sides.  Everything is
built for the shifted operator A_alpha (eq. helmalpha).

Readings (also listed in the design notes):
* middle subproblem = 2B-1 rows c-B+1 .. c+B-1, damped towards both ends;
* c = (n+1)/2 for odd n and n/2+1 for even n;
* the coupling A_{m+1,m} used between layers is the physical one (a block of A_alpha);
* ``exact=True`` replaces every subproblem by the true principal block of
  A_alpha seen by that layer at its turn in the elimination order (rows 1..m
  for the lower front, m..n for the upper front, all rows for the middle).
  Then each T~ equals the exact Schur inverse of eq. Afactm and the operator
  is A_alpha^{-1} exactly -- the identity used to pin this module.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
from scipy.linalg import lapack

from .helmholtz import (Params, sigma_low, sigma_phys, stretch, strip_operator, x1_profiles,
                        x2_phys_profiles, row_coupling)


@dataclass
class SubSpec:
    """One subproblem: its physical rows (increasing) and the x2 damping at rows and half rows."""
    kind: str                 # 'F', 'E', 'lower', 'upper', 'mid'
    m: int                    # layer index (for F: B, for E: n-B+1)
    rows: np.ndarray          # 1-based physical rows, increasing
    sig_node: np.ndarray      # sigma at the rows
    sig_half: np.ndarray      # sigma at the len(rows)+1 half rows
    slot: int                 # local (0-based) index of the layer row inside ``rows``
    full: bool                # F / E: input and output on all rows


def _spec_moving_lower(p: Params, m: int) -> SubSpec:
    """Layer m of the upward front: rows m-B+1..m, sigma_2 measured from (m-B)h (Section 2.2)."""
    B, h, C, eta = p.B, p.h, p.C, p.eta_move
    rows = np.arange(m - B + 1, m + 1)
    t_node = h * rows - (m - B) * h
    t_half = h * (np.arange(m - B, m + 1) + 0.5) - (m - B) * h
    return SubSpec('lower', m, rows, sigma_low(t_node, eta, C), sigma_low(t_half, eta, C), B - 1, False)


def _spec_moving_upper(p: Params, m: int) -> SubSpec:
    """Layer m of the downward front: rows m..m+B-1, damping measured from (m+B)h downwards."""
    B, h, C, eta = p.B, p.h, p.C, p.eta_move
    rows = np.arange(m, m + B)
    t_node = (m + B) * h - h * rows
    t_half = (m + B) * h - h * (np.arange(m - 1, m + B) + 0.5)
    return SubSpec('upper', m, rows, sigma_low(t_node, eta, C), sigma_low(t_half, eta, C), 0, False)


def _spec_middle(p: Params, c: int) -> SubSpec:
    """Middle layer c with moving PMLs on both sides: rows c-B+1..c+B-1."""
    B, h, C, eta = p.B, p.h, p.C, p.eta_move
    rows = np.arange(c - B + 1, c + B)
    x_node = h * rows
    x_half = h * (np.arange(c - B, c + B) + 0.5)
    sn = sigma_low(x_node - (c - B) * h, eta, C) + sigma_low((c + B) * h - x_node, eta, C)
    shf = sigma_low(x_half - (c - B) * h, eta, C) + sigma_low((c + B) * h - x_half, eta, C)
    return SubSpec('mid', c, rows, sn, shf, B - 1, False)


def _spec_phys(p: Params, kind: str, m: int, rows: np.ndarray, slot: int, full: bool) -> SubSpec:
    """A principal block of A_alpha: physical x2 damping on consecutive rows."""
    h = p.h
    t_node = h * rows
    t_half = h * (np.arange(rows[0] - 1, rows[-1] + 1) + 0.5)
    return SubSpec(kind, m, rows, sigma_phys(t_node, p.eta_phys, p.C),
                   sigma_phys(t_half, p.eta_phys, p.C), slot, full)


def subproblem_specs(p: Params, exact: bool = False) -> Dict:
    """All subproblems of the two-front sweep, in elimination order per front."""
    n, B, c = p.n, p.B, p.mid
    if n < 2 * B + 3:
        raise ValueError(f"n={n} too small for B={B}: need n >= 2B+3")
    F = _spec_phys(p, 'F', B, np.arange(1, B + 1), B - 1, True)
    E = _spec_phys(p, 'E', n - B + 1, np.arange(n - B + 1, n + 1), 0, True)
    lower, upper = [], []
    for m in range(B + 1, c):
        if exact:
            lower.append(_spec_phys(p, 'lower', m, np.arange(1, m + 1), m - 1, False))
        else:
            lower.append(_spec_moving_lower(p, m))
    for m in range(n - B, c, -1):
        if exact:
            upper.append(_spec_phys(p, 'upper', m, np.arange(m, n + 1), 0, False))
        else:
            upper.append(_spec_moving_upper(p, m))
    if exact:
        mid = _spec_phys(p, 'mid', c, np.arange(1, n + 1), c - 1, False)
    else:
        mid = _spec_middle(p, c)
    return {'F': F, 'E': E, 'lower': lower, 'upper': upper, 'mid': mid}


def sub_operator(p: Params, c: np.ndarray, spec: SubSpec):
    """H on the subproblem's strip in row-by-row order (eq. helma discretised like eq. helmd)."""
    n = p.n
    c2 = np.asarray(c, dtype=np.float64).reshape(n, n)
    s1n, s1h = x1_profiles(p)
    s2n = stretch(spec.sig_node, p.omega)
    s2h = stretch(spec.sig_half, p.omega)
    kappa = p.omega + 1j * p.alpha
    return strip_operator(c2[spec.rows - 1, :], p.h, s1n, s1h, s2n, s2h, kappa)


@dataclass
class BandLU:
    """LAPACK band LU of P H P^t (x2-first ordering, half-bandwidth R = number of rows)."""
    spec: SubSpec
    R: int
    n: int
    lu: np.ndarray
    ipiv: np.ndarray

    def solve_rows(self, g_rows: np.ndarray) -> np.ndarray:
        """H^{-1} g for g given as (R, n, k) in strip row order; returns (R, n, k)."""
        R, n = self.R, self.n
        k = g_rows.shape[2]
        # x2-first ordering: local index (i-1)*R + r
        b = np.ascontiguousarray(np.transpose(g_rows, (1, 0, 2)).reshape(n * R, k))
        x, info = lapack.zgbtrs(self.lu, R, R, b, self.ipiv)
        if info != 0:
            raise RuntimeError(f"zgbtrs info={info}")
        return np.transpose(x.reshape(n, R, k), (1, 0, 2))


def band_factor(p: Params, c: np.ndarray, spec: SubSpec) -> BandLU:
    """Permute H to the x2-first ordering (Section 2.2) and factor it with zgbtrf, kl = ku = R."""
    H = sub_operator(p, c, spec).tocoo()
    R, n = len(spec.rows), p.n
    # row-major strip index r*n + (i-1)  ->  x2-first index (i-1)*R + r
    def perm(idx):
        r, i = np.divmod(idx, n)
        return i * R + r
    ri, ci = perm(H.row), perm(H.col)
    kl = ku = R
    N = R * n
    ab = np.zeros((2 * kl + ku + 1, N), dtype=np.complex128)
    ab[kl + ku + ri - ci, ci] = H.data
    lu, ipiv, info = lapack.zgbtrf(ab, kl, ku)
    if info != 0:
        raise RuntimeError(f"zgbtrf info={info} ({spec.kind} m={spec.m})")
    return BandLU(spec, R, n, lu, ipiv)


@dataclass
class SweepFactor:
    """Algorithm 3 output: band LU factors of F, E, every moving layer and the middle."""
    p: Params
    F: BandLU
    E: BandLU
    lower: List[BandLU]
    upper: List[BandLU]
    mid: BandLU
    exact: bool = False
    cpl: Dict[int, np.ndarray] = field(default_factory=dict)

    def coupling(self, j: int) -> np.ndarray:
        """Diagonal of A_{j+1,j} (rows j and j+1)."""
        if j not in self.cpl:
            self.cpl[j] = row_coupling(self.p, j)
        return self.cpl[j]


def factor(p: Params, c: np.ndarray, exact: bool = False) -> SweepFactor:
    """Algorithm 3 with two fronts: factor every subproblem of the sweep."""
    specs = subproblem_specs(p, exact)
    return SweepFactor(p,
                       band_factor(p, c, specs['F']), band_factor(p, c, specs['E']),
                       [band_factor(p, c, s) for s in specs['lower']],
                       [band_factor(p, c, s) for s in specs['upper']],
                       band_factor(p, c, specs['mid']), exact)


def _T_slot(sub: BandLU, g: np.ndarray) -> np.ndarray:
    """T~ g: load g (n, k) on the layer row, return the solution on the layer row."""
    rhs = np.zeros((sub.R, sub.n, g.shape[1]), dtype=np.complex128)
    rhs[sub.spec.slot] = g
    return sub.solve_rows(rhs)[sub.spec.slot]


def _T_slot_full(sub: BandLU, g: np.ndarray) -> np.ndarray:
    """Load g on the layer row, return the solution on every row of the subproblem (F / E)."""
    rhs = np.zeros((sub.R, sub.n, g.shape[1]), dtype=np.complex128)
    rhs[sub.spec.slot] = g
    return sub.solve_rows(rhs)


def apply_sweep(M: SweepFactor, f: np.ndarray) -> np.ndarray:
    """Algorithm 4, two-front form: u = M_alpha f.

    f has shape (n*n,) or (k, n*n) (k right-hand sides); the result has the same shape.
    """
    p = M.p
    n, B, c = p.n, p.B, p.mid
    single = (f.ndim == 1)
    F2 = np.atleast_2d(np.asarray(f, dtype=np.complex128))
    k = F2.shape[0]
    U = np.transpose(F2.reshape(k, n, n), (1, 2, 0)).copy()   # U[j-1] = u_j, shape (n, n, k)
    Y = np.zeros_like(U)
    a = M.coupling

    # forward substitution + diagonal applications, upward front: F, B+1, ..., c-1
    Y[0:B] = M.F.solve_rows(U[0:B])
    U[B] -= a(B)[:, None] * Y[B - 1]
    for sub in M.lower:
        m = sub.spec.m
        Y[m - 1] = _T_slot(sub, U[m - 1])
        U[m] -= a(m)[:, None] * Y[m - 1]
    # downward front: E, n-B, ..., c+1
    Y[n - B:n] = M.E.solve_rows(U[n - B:n])
    U[n - B - 1] -= a(n - B)[:, None] * Y[n - B]
    for sub in M.upper:
        m = sub.spec.m
        Y[m - 1] = _T_slot(sub, U[m - 1])
        U[m - 2] -= a(m - 1)[:, None] * Y[m - 1]
    # middle layer, after both fronts have updated it
    Y[c - 1] = _T_slot(M.mid, U[c - 1])

    # backward substitution, upward front in reverse: c-1, ..., B+1, then F
    for sub in reversed(M.lower):
        m = sub.spec.m
        Y[m - 1] -= _T_slot(sub, a(m)[:, None] * Y[m])
    Y[0:B] -= _T_slot_full(M.F, a(B)[:, None] * Y[B])
    # downward front in reverse: c+1, ..., n-B, then E
    for sub in reversed(M.upper):
        m = sub.spec.m
        Y[m - 1] -= _T_slot(sub, a(m - 1)[:, None] * Y[m - 2])
    Y[n - B:n] -= _T_slot_full(M.E, a(n - B)[:, None] * Y[n - B - 1])

    out = np.transpose(Y, (2, 0, 1)).reshape(k, n * n)
    return out[0] if single else out


def T_tilde_matrix(sub: BandLU) -> np.ndarray:
    """Dense n x n matrix of T~ (layer row in, layer row out), column by column."""
    return _T_slot(sub, np.eye(sub.n, dtype=np.complex128))
