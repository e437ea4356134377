"""Pins of the oracle's sweeping preconditioner (Sections 2.1-2.3, Algorithms 1-4)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import exact as X
from oracle import helmholtz as H
from oracle import krylov as K
from oracle import sweep as S


def _setup(n, w=4, freq=3.0, field="lens", alpha=2.0, seed=0):
    par = H.Params(n=n, omega=2 * math.pi * freq, alpha=alpha, pml_w=w, mpml_w=w)
    if field == "lens":
        c = workloads.velocity_lens(n)
    elif field == "grf":
        c = workloads.velocity_grf(n, seed=seed + 11)
    else:
        c = workloads.velocity_const(n)
    return par, c


def test_band_lu_matches_dense_inverse():
    """T~ through the permuted LAPACK band LU equals the layer-row block of the dense H^{-1} (Section 2.2)."""
    par, c = _setup(19, w=3, field="grf")
    specs = S.subproblem_specs(par)
    subs = [specs['F'], specs['E'], specs['mid'], specs['lower'][0], specs['lower'][-1],
            specs['upper'][0], specs['upper'][-1]]
    rng = np.random.default_rng(2)
    n = par.n
    for spec in subs:
        Hs = S.sub_operator(par, c, spec).toarray()
        R = len(spec.rows)
        g = rng.standard_normal((R, n, 2)) + 1j * rng.standard_normal((R, n, 2))
        lu = S.band_factor(par, c, spec)
        x = lu.solve_rows(g)
        xd = np.linalg.solve(Hs, g.reshape(R * n, 2)).reshape(R, n, 2)
        np.testing.assert_allclose(x, xd, rtol=0, atol=1e-11 * np.abs(xd).max())


def test_front_block_is_principal_block_of_A_alpha():
    """Algorithm 3, step 1: H_F = A_{F,F} (and likewise H_E = A_{E,E})."""
    par, c = _setup(21, w=4, field="grf")
    A = H.assemble(par, c, shifted=True).toarray()
    specs = S.subproblem_specs(par)
    n, B = par.n, par.B
    HF = S.sub_operator(par, c, specs['F']).toarray()
    HE = S.sub_operator(par, c, specs['E']).toarray()
    np.testing.assert_array_equal(HF, A[:B * n, :B * n])
    np.testing.assert_array_equal(HE, A[(n - B) * n:, (n - B) * n:])


@pytest.mark.parametrize("n,field,pw", [(21, "lens", 3), (22, "grf", 3), (31, "grf", 3), (27, "const", 3),
                                         (29, "grf", 7), (26, "lens", 6)])
def test_exact_mode_is_inverse_of_A_alpha(n, field, pw):
    """Eq. Afactm: with every subproblem the true principal block, T~_m = S_m^{-1} and the two-front
    sweep reproduces A_alpha^{-1} (sparse direct solve as the reference).  pw > 3 puts physical
    damping into the couplings between the first layers of each front."""
    par, c = _setup(n, w=3, field=field)
    par = H.Params(n=par.n, omega=par.omega, alpha=par.alpha, pml_w=pw, mpml_w=3)
    Aa = H.assemble(par, c, shifted=True).tocsc()
    M = S.factor(par, c, exact=True)
    f = workloads.random_rhs(n, 3, seed=n)
    u = S.apply_sweep(M, f)
    for k in range(3):
        ud = spla.spsolve(Aa, f[k])
        assert np.linalg.norm(u[k] - ud) <= 1e-11 * np.linalg.norm(ud)


def test_algorithms_1_2_dense_exact():
    """Algorithms 1 and 2 (dense T_m) give u = A^{-1} f."""
    par, c = _setup(17, w=3, field="grf")
    n = par.n
    A = H.assemble(par, c)
    T = X.setup_exact(A, n)
    f = workloads.random_rhs(n, 1, 5)[0]
    u = X.solve_exact(A, n, T, f)
    ud = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(u - ud) <= 1e-11 * np.linalg.norm(ud)


def test_exact_preconditioner_one_iteration_alpha0():
    """alpha = 0 and exact subproblems: M = A^{-1}, so FGMRES stops after one iteration."""
    par, c = _setup(25, w=3, field="lens", alpha=0.0)
    A = H.assemble(par, c)
    M = S.factor(par, c, exact=True)
    f = workloads.source_point_at(25, 0.5, 0.3)
    r = K.fgmres(lambda v: A @ v, lambda v: S.apply_sweep(M, v), f, restart=10, tol=1e-10)
    assert r.converged and r.iters == 1 and r.relres < 1e-10


@pytest.mark.parametrize("n", [23, 30])
def test_preconditioner_complex_symmetric(n):
    """M_alpha = L^{-t} D^{-1} L^{-1} with symmetric T~: x^t M y = y^t M x (no conjugation)."""
    par, c = _setup(n, w=4, field="grf")
    M = S.factor(par, c)
    x, y = workloads.random_rhs(n, 2, seed=3 + n)
    a = x @ S.apply_sweep(M, y)
    b = y @ S.apply_sweep(M, x)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_T_tilde_symmetric():
    """Each T~_m is complex symmetric (H_m is)."""
    par, c = _setup(21, w=4, field="grf")
    M = S.factor(par, c)
    for sub in (M.lower[1], M.upper[2], M.mid):
        T = S.T_tilde_matrix(sub)
        np.testing.assert_allclose(T, T.T, rtol=0, atol=1e-12 * np.abs(T).max())


@pytest.mark.parametrize("kind", ["lower", "upper", "mid"])
def test_moving_pml_converges_to_exact_schur_inverse(kind):
    """Section 2.2: T~_m approximates T_m = S_m^{-1}; the approximation improves as the moving PML
    widens (fixed grid, fixed layer).  A damping profile on the wrong side of the strip, or a wrong
    sign, breaks the trend."""
    n, freq = 45, 4.0
    errs = []
    for w in (2, 5, 11):
        par = H.Params(n=n, omega=2 * math.pi * freq, alpha=2.0, pml_w=2, mpml_w=w)
        c = workloads.velocity_const(n)
        ex = S.subproblem_specs(par, exact=True)
        mv = S.subproblem_specs(par)
        m = par.mid - 3 if kind == "lower" else par.mid + 3
        pick = {'lower': lambda d: [s for s in d['lower'] if s.m == m][0],
                'upper': lambda d: [s for s in d['upper'] if s.m == m][0],
                'mid': lambda d: d['mid']}[kind]
        Te = S.T_tilde_matrix(S.band_factor(par, c, pick(ex)))
        Tm = S.T_tilde_matrix(S.band_factor(par, c, pick(mv)))
        # compare away from the physical x1 PML
        sl = slice(8, n - 8)
        errs.append(np.linalg.norm((Tm - Te)[sl, sl]) / np.linalg.norm(Te[sl, sl]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


@pytest.mark.parametrize("n,pw,mw", [(31, 4, 4), (30, 4, 4), (33, 7, 3)])
def test_mirror_symmetry_of_two_front_sweep(n, pw, mw):
    """For c symmetric under x2 -> 1 - x2 the continuous problem, the PML of eq. sigma and the
    two-front construction are mirror symmetric (the downward front is the upward one reflected,
    the middle layer is damped alike on both sides), so M_alpha commutes with the row reflection.
    Likewise with the column reflection for c symmetric in x1."""
    par = H.Params(n=n, omega=2 * math.pi * 3, alpha=2.0, pml_w=pw, mpml_w=mw)
    c = workloads.velocity_lens(n)                      # symmetric in x1 and in x2
    if n % 2 == 0:
        return _mirror_even(par, c)
    M = S.factor(par, c)
    f = workloads.random_rhs(n, 2, seed=n)
    flip_rows = lambda v: v.reshape(-1, n, n)[:, ::-1, :].reshape(v.shape)
    flip_cols = lambda v: v.reshape(-1, n, n)[:, :, ::-1].reshape(v.shape)
    for flip in (flip_rows, flip_cols):
        a = S.apply_sweep(M, flip(f))
        b = flip(S.apply_sweep(M, f))
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def _mirror_even(par, c):
    """Even n has no middle row (c = n/2+1 is off-centre), so only the column reflection applies."""
    n = par.n
    M = S.factor(par, c)
    f = workloads.random_rhs(n, 1, seed=n)
    flip_cols = lambda v: v.reshape(-1, n, n)[:, :, ::-1].reshape(v.shape)
    a = S.apply_sweep(M, flip_cols(f))
    b = flip_cols(S.apply_sweep(M, f))
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("mw", [2, 4, 6])
def test_middle_strip_damped_alike_on_both_sides(mw):
    """The middle layer has moving PMLs on both sides (two-front sweep, Section 2.3): for c symmetric
    about the middle row its strip operator is invariant under the reflection of its 2B-1 rows, and the
    lower / upper moving strips of mirrored layers are reflections of each other."""
    n = 31
    par = H.Params(n=n, omega=2 * math.pi * 3, alpha=2.0, pml_w=3, mpml_w=mw)
    c = workloads.velocity_lens(n)
    specs = S.subproblem_specs(par)
    Hm = S.sub_operator(par, c, specs['mid']).toarray()
    R = len(specs['mid'].rows)
    assert R == 2 * par.B - 1
    P = np.arange(R * n).reshape(R, n)[::-1, :].ravel()
    np.testing.assert_allclose(Hm, Hm[np.ix_(P, P)], rtol=1e-13, atol=1e-13 * np.abs(Hm).max())
    for lo in specs['lower']:
        up = [s for s in specs['upper'] if s.m == n + 1 - lo.m][0]
        Hl = S.sub_operator(par, c, lo).toarray()
        Hu = S.sub_operator(par, c, up).toarray()
        Pb = np.arange(par.B * n).reshape(par.B, n)[::-1, :].ravel()
        np.testing.assert_allclose(Hu, Hl[np.ix_(Pb, Pb)], rtol=1e-13, atol=1e-13 * np.abs(Hl).max())


@pytest.mark.parametrize("n,w", [(29, 4), (30, 3), (41, 6)])
def test_moving_strips_equal_front_blocks_for_x2_independent_c(n, w):
    """Section 2.2, s2^m(x2) = s(sigma_2(x2 - (m - b)h)): the moving PML of layer m is the physical
    bottom PML shifted up to the strip.  With equal physical and moving widths and a velocity that
    does not depend on x2, every lower strip operator H_m is therefore entry for entry the front block
    A_alpha[F, F], and every upper one A_alpha[E, E].  An offset of one row in either front's
    profile (a consistent off-by-one keeps the monotone-trend and mirror pins) breaks this."""
    par = H.Params(n=n, omega=2 * math.pi * 3.5, alpha=2.0, pml_w=w, mpml_w=w)
    # c depends on x1 only: the same row repeated
    c = np.tile(workloads.velocity_waveguide(n, seed=3).reshape(n, n)[n // 2], (n, 1)).ravel()
    A = H.assemble(par, c, shifted=True).toarray()
    B = par.B
    AF = A[:B * n, :B * n]
    AE = A[(n - B) * n:, (n - B) * n:]
    specs = S.subproblem_specs(par)
    assert len(specs['lower']) > 2 and len(specs['upper']) > 2
    for spec in specs['lower']:
        Hm = S.sub_operator(par, c, spec).toarray()
        np.testing.assert_allclose(Hm, AF, rtol=1e-13, atol=1e-13 * np.abs(AF).max())
    for spec in specs['upper']:
        Hm = S.sub_operator(par, c, spec).toarray()
        np.testing.assert_allclose(Hm, AE, rtol=1e-13, atol=1e-13 * np.abs(AE).max())


def test_b_convention_literal_is_a_relabelling():
    """The paper-literal width convention (eta = w h, B = w) with width w + 1 builds the same PMLs and
    strips as the default (eta = (w + 1) h, B = w + 1) with width w: equal B, eta and M_alpha."""
    n, w = 33, 4
    p0 = H.Params(n=n, omega=2 * math.pi * 3, alpha=2.0, pml_w=w, mpml_w=w, b_convention=0)
    p1 = H.Params(n=n, omega=2 * math.pi * 3, alpha=2.0, pml_w=w + 1, mpml_w=w + 1, b_convention=1)
    assert p0.B == p1.B == w + 1
    assert p0.eta_phys == p1.eta_phys and p0.eta_move == p1.eta_move
    c = workloads.velocity_grf(n, seed=8)
    f = workloads.random_rhs(n, 2, seed=9)
    u0 = S.apply_sweep(S.factor(p0, c), f)
    u1 = S.apply_sweep(S.factor(p1, c), f)
    np.testing.assert_array_equal(u0, u1)
    # and the literal convention is itself exact in exact mode (its B = w strips, eta = w h)
    p2 = H.Params(n=n, omega=2 * math.pi * 3, alpha=2.0, pml_w=w, mpml_w=w, b_convention=1)
    assert p2.B == w and abs(p2.eta_move - w * p2.h) < 1e-15
    Aa = H.assemble(p2, c, shifted=True).tocsc()
    u2 = S.apply_sweep(S.factor(p2, c, exact=True), f)
    for k in range(2):
        ud = spla.spsolve(Aa, f[k])
        assert np.linalg.norm(u2[k] - ud) <= 1e-11 * np.linalg.norm(ud)
