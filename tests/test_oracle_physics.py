"""Physical pins: the discrete solution converges to the free-space Green's function at second order,
and the Green's function is reciprocal (A = A^t)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import scipy.special as ss

import workloads
from oracle import helmholtz as H
from oracle import krylov as K
from oracle import sweep as S


def _hankel_error(n, eta_rows, omega):
    par = H.Params(n=n, omega=omega, pml_w=eta_rows - 1, mpml_w=eta_rows - 1)
    f = workloads.source_point_at(n, 0.5, 0.5)
    u = spla.spsolve(H.assemble(par, workloads.velocity_const(n)).tocsc(), f)
    X1, X2, _ = workloads.grid(n)
    x1, x2 = X1.ravel(), X2.ravel()
    r = np.hypot(x1 - 0.5, x2 - 0.5)
    G = -0.25j * ss.hankel1(0, omega * r)          # (Laplacian + omega^2) G = delta, outgoing
    eta = par.eta_phys
    mask = (r > 0.1) & (np.minimum.reduce([x1, x2, 1 - x1, 1 - x2]) > eta)
    return np.linalg.norm(u[mask] - G[mask]) / np.linalg.norm(G[mask])


@pytest.mark.slow
def test_point_source_converges_to_hankel_second_order():
    """Constant c, unit-mass point source: error against -(i/4) H_0^(1)(omega r) away from the source and
    the PML falls by ~4 per halving of h (fixed physical PML width).  Pins the PML sign (outgoing,
    absorbing), the stencil and the source scaling together."""
    omega = 2 * math.pi * 4
    e = [_hankel_error(n, r, omega) for n, r in [(63, 9), (127, 18), (255, 36)]]
    assert 3.5 < e[0] / e[1] < 4.5
    assert 3.5 < e[1] / e[2] < 4.5
    assert e[2] < 5e-3


def test_point_source_hankel_coarse():
    """Fast variant of the Hankel pin (two grids)."""
    omega = 2 * math.pi * 3
    e1 = _hankel_error(47, 8, omega)
    e2 = _hankel_error(95, 16, omega)
    assert 3.3 < e1 / e2 < 4.7


def test_reciprocity_direct_and_preconditioned():
    """G(x, y) = G(y, x): the response at y to a source at x equals the response at x to a source at y,
    both with the sparse direct solve (1e-12) and with preconditioned FGMRES (1e-5)."""
    n = 47
    par = H.Params(n=n, omega=2 * math.pi * 5, pml_w=6, mpml_w=6)
    c = workloads.velocity_grf(n, seed=31)
    A = H.assemble(par, c)
    ix, jx, iy, jy = 12, 30, 35, 14
    fx = workloads.source_point(n, ix, jx)
    fy = workloads.source_point(n, iy, jy)
    px, py = (jx - 1) * n + ix - 1, (jy - 1) * n + iy - 1
    ux = spla.spsolve(A.tocsc(), fx)
    uy = spla.spsolve(A.tocsc(), fy)
    assert abs(ux[py] - uy[px]) <= 1e-12 * abs(ux[py])
    M = S.factor(par, c)
    rx = K.fgmres(lambda v: A @ v, lambda v: S.apply_sweep(M, v), fx, 20, 1e-9)
    ry = K.fgmres(lambda v: A @ v, lambda v: S.apply_sweep(M, v), fy, 20, 1e-9)
    assert abs(rx.x[py] - ry.x[px]) <= 1e-5 * abs(ux[py])
