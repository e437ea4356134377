"""Pins of the oracle's operator (eq. sigma, eq. helmd, eq. helmalpha) against facts that do not
come from the oracle itself: textbook eigenpairs, exact symmetry, a separable 1D reduction."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import helmholtz as H


def _params(n, omega, C=20.0, w=4, alpha=2.0):
    return H.Params(n=n, omega=omega, alpha=alpha, pml_w=w, mpml_w=w, C=C)


@pytest.mark.parametrize("n", [15, 24, 31])
def test_operator_complex_symmetric_bitwise(n):
    """Section 2.1: the stretched form is chosen for its symmetry; A = A^t exactly (no conjugation)."""
    rng = np.random.default_rng(n)
    c = rng.uniform(0.7, 1.4, n * n)
    for shifted in (False, True):
        A = H.assemble(_params(n, 2 * math.pi * 3), c, shifted=shifted)
        D = (A - A.T).tocoo()
        assert D.nnz == 0 or np.max(np.abs(D.data)) == 0.0
        # block structure: A_{m,m} tridiagonal, A_{m,m+1} diagonal (Section 2.1)
        Ad = A.toarray()
        off = Ad[0:n, n:2 * n]
        assert np.count_nonzero(off - np.diag(np.diag(off))) == 0
        blk = Ad[n:2 * n, n:2 * n]
        assert np.count_nonzero(np.triu(blk, 2)) == 0 and np.count_nonzero(np.tril(blk, -2)) == 0


@pytest.mark.parametrize("n,p,q", [(15, 1, 1), (15, 3, 7), (20, 2, 5), (31, 11, 4)])
def test_no_pml_constant_c_eigenpairs(n, p, q):
    """C = 0, c = 1: the textbook 5-point Laplacian plus omega^2.  v_ij = sin(p pi i h) sin(q pi j h),
    lambda = omega^2 - (4/h^2)(sin^2(p pi h/2) + sin^2(q pi h/2))."""
    omega = 2 * math.pi * 2.5
    par = _params(n, omega, C=0.0)
    A = H.assemble(par, workloads.velocity_const(n))
    h = par.h
    i = np.arange(1, n + 1)
    v = np.outer(np.sin(q * math.pi * i * h), np.sin(p * math.pi * i * h)).ravel()  # [j, i]
    lam = omega ** 2 - (4 / h ** 2) * (math.sin(p * math.pi * h / 2) ** 2 + math.sin(q * math.pi * h / 2) ** 2)
    np.testing.assert_allclose(A @ v, lam * v, rtol=0, atol=1e-9 * abs(lam) * np.abs(v).max())


def test_no_pml_shift_is_scalar_mass():
    """C = 0: A_alpha - A = ((omega + i alpha)^2 - omega^2) / c^2 on the diagonal only (eq. helmalpha)."""
    n = 17
    rng = np.random.default_rng(1)
    c = rng.uniform(0.8, 1.5, n * n)
    par = _params(n, 2 * math.pi * 2, C=0.0, alpha=2.0)
    D = (H.assemble(par, c, shifted=True) - H.assemble(par, c)).toarray()
    expect = ((par.omega + 2.0j) ** 2 - par.omega ** 2) / c ** 2
    np.testing.assert_allclose(np.diag(D), expect, rtol=1e-12)
    assert np.count_nonzero(D - np.diag(np.diag(D))) == 0


def test_layered_medium_separable_eigenpairs():
    """C = 0 and c = c(x2): A separates into sin modes in x1 times eigenvectors of the 1D problem
    (1/h^2) tridiag(1,-2,1) + diag(omega^2 / c_j^2) in x2 (scipy eigh_tridiagonal).  Pins the
    orientation of c and of the row-by-row ordering."""
    n = 21
    c = workloads.velocity_layered(n, seed=7)
    assert np.ptp(c.reshape(n, n)[:, 0]) > 0.1           # really varies along x2
    omega = 2 * math.pi * 3
    par = _params(n, omega, C=0.0)
    A = H.assemble(par, c)
    h = par.h
    cj = c.reshape(n, n)[:, 0]
    d = -2 / h ** 2 + omega ** 2 / cj ** 2
    e = np.full(n - 1, 1 / h ** 2)
    mu, psi = sla.eigh_tridiagonal(d, e)
    i = np.arange(1, n + 1)
    for p, k in [(1, 0), (4, 9), (13, 20)]:
        v = np.outer(psi[:, k], np.sin(p * math.pi * i * h)).ravel()
        lam = mu[k] - (4 / h ** 2) * math.sin(p * math.pi * h / 2) ** 2
        np.testing.assert_allclose(A @ v, lam * v, rtol=0, atol=1e-8 * np.abs(lam))


def test_sigma_profile_shape():
    """eq. sigma: zero on the undamped part, largest (C/eta) at the outer boundary, quadratic."""
    eta, C = 0.25, 20.0
    t = np.array([0.0, eta / 2, eta, 0.5, 1 - eta, 1 - eta / 2, 1.0])
    s = H.sigma_phys(t, eta, C)
    np.testing.assert_allclose(s, [C / eta, C / eta / 4, 0, 0, 0, C / eta / 4, C / eta], rtol=1e-14)
    # the stretch damps outgoing waves e^{i omega x}: |s| < 1, Im s < 0 where sigma > 0
    st = H.stretch(np.array([0.0, 3.0]), 5.0)
    assert st[0] == 1.0 and abs(st[1]) < 1.0 and st[1].imag < 0.0
