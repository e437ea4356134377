"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, element by element.

Every comparison is entry-wise (tests/parity_util.py): max |gpu - oracle| / max |oracle| over the
output, and for preconditioner applications also inside every grid row and every 16-column block of a
row, so that errors in small-magnitude rows (PML, F / E strips) or in the ragged last segment show.

Tolerances (entry-wise):
  matvec 1e-14 (five FP64 products per entry);
  FP64 strip solve 1e-11 and sweep 1e-11 (u = 1.1e-16 through an n-column block recurrence per strip
  and ~n strips per front; observed at most 1e-13 entry-wise), row-wise 1e-10 (observed 7e-13);
  complex64 factors: strip solve 2e-5, sweep tol_c64(n) below (u = 6e-8 times the growth of the block
  recurrences, linear in n);
FGMRES: the solution agrees with the oracle's to 1e-6 relative (both stop at a 1e-6 true residual on
the same Krylov sequence).
"""
import math
import sys

import numpy as np
import pytest

import workloads
from parity_util import col_seg_rel, elem_rel, row_rel
from oracle import helmholtz as OH
from oracle import krylov as OK
from oracle import sweep as OS

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hs():
    from paper_1007_4291_amd import helmsweep
    return helmsweep


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _case(name):
    """(oracle params, c, gpu params) for small parity cases."""
    if name == "cfg1":
        pr = workloads.cfg1()
        c, n, om, w = pr.c, pr.n, pr.omega, 8
        pw = w
    elif name == "grf45":
        n, om, w, pw = 45, 2 * math.pi * 5, 4, 4
        c = workloads.velocity_grf(n, seed=77)
    elif name == "even40":
        n, om, w, pw = 40, 2 * math.pi * 4, 3, 6
        c = workloads.velocity_lens(n)
    elif name == "lens61w12":
        n, om, w, pw = 61, 2 * math.pi * 6, 12, 12
        c = workloads.velocity_lens(n)
    elif name == "wg71w16":
        n, om, w, pw = 71, 2 * math.pi * 7, 16, 16
        c = workloads.velocity_waveguide(n, seed=5)
    else:
        raise KeyError(name)
    op = OH.Params(n=n, omega=om, alpha=2.0, pml_w=pw, mpml_w=w)
    return op, c


def _gpu_problem(hs, torch, op, c):
    gp = hs.Params(n=op.n, omega=op.omega, alpha=op.alpha, pml_w=op.pml_w, mpml_w=op.mpml_w, C=op.C)
    return hs.Problem(gp, torch.as_tensor(c, dtype=torch.float64, device="cuda"))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


TOL_C128 = (1e-11, 1e-10)     # sweep apply: entry-wise, row-wise (observed <= 1e-13 / 7e-13)
TOL_C64 = "c64"               # n-dependent, tol_c64(n)
FLOOR = 1e-2                  # rows / blocks below 1e-2 of the output's maximum: see parity_util


def tol_c64(n):
    """complex64 factors and FP32 sweep: the rounding error grows about linearly with the length of the
    column recurrences and the number of layers (observed entry-wise 3e-7 at n = 63, 1.5e-6 at n = 255,
    4.9e-6 at n = 511; row / block-wise 2.4e-5 at n = 511): 4e-8 n entry-wise, 4e-7 n row-wise, with
    floors 2e-6 / 2e-5 -- a margin of 4-8x over every observation."""
    return (max(2e-6, 4e-8 * n), max(2e-5, 4e-7 * n))


def _check_apply(u, uo, n, tol, label=""):
    """Entry-wise, row-wise and 16-column-block-wise parity of a preconditioner application."""
    if tol == TOL_C64:
        tol = tol_c64(n)
    e, r, c = elem_rel(u, uo), row_rel(u, uo, n, FLOOR), col_seg_rel(u, uo, n, 16, FLOOR)
    _log(f"  {label} entry {e:.2e} row {r:.2e} colseg {c:.2e} (norm {_rel(u, uo):.2e})")
    assert e <= tol[0], (label, e)
    assert r <= tol[1] and c <= tol[1], (label, r, c)


@pytest.mark.parametrize("name", ["cfg1", "even40", "wg71w16"])
def test_matvec_parity(hs, torch, name):
    op, c = _case(name)
    _log("matvec", name)
    A = _gpu_problem(hs, torch, op, c)
    Ao = OH.assemble(op, c)
    x = workloads.random_rhs(op.n, 3, seed=1)
    y = A.matvec(torch.as_tensor(x, device="cuda")).cpu().numpy()
    for k in range(3):
        assert elem_rel(y[k], Ao @ x[k]) <= 1e-14
    x32 = torch.as_tensor(x, device="cuda").to(torch.complex64)
    y32 = A.matvec(x32).cpu().numpy()
    xr = x32.cpu().numpy().astype(np.complex128)
    for k in range(3):
        assert elem_rel(y32[k], Ao @ xr[k]) <= 1e-14


def _sub_map(op, M, sub):
    """GPU strip index -> (oracle BandLU, local->oracle row permutation)."""
    L_lo = op.mid - 1 - op.B
    if sub == 0:
        return M.F, None
    if sub <= L_lo:
        return M.lower[sub - 1], None
    if sub == L_lo + 1:
        return M.E, "flip"
    nsub = len(M.lower) + len(M.upper) + 3
    if sub == nsub - 1:
        return M.mid, None
    return M.upper[sub - L_lo - 2], "flip"


@pytest.mark.parametrize("name,prec", [("cfg1", 0), ("grf45", 0), ("even40", 0), ("wg71w16", 0),
                                       ("cfg1", 1), ("lens61w12", 1)])
def test_strip_solve_parity(hs, torch, name, prec):
    """Each strip's block LU solve (a2 factor + one solve) equals the oracle's LAPACK band solve."""
    op, c = _case(name)
    _log("strip", name, prec)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, prec)
    Mo = OS.factor(op, c)
    nsub = F.num_subproblems
    assert nsub == len(Mo.lower) + len(Mo.upper) + 3
    L_lo = op.mid - 1 - op.B
    picks = sorted(set([0, 1, L_lo, L_lo + 1, L_lo + 2, nsub - 2, nsub - 1]))
    tol = 1e-11 if prec == 0 else 2e-5
    rng = np.random.default_rng(3)
    for sub in picks:
        band, flip = _sub_map(op, Mo, sub)
        R = F.subproblem_rows(sub)
        assert R == band.R
        g = rng.standard_normal((5, R, op.n)) + 1j * rng.standard_normal((5, R, op.n))
        x = F.subsolve(sub, torch.as_tensor(g, device="cuda")).cpu().numpy()
        go = g[:, ::-1, :] if flip else g
        xo = band.solve_rows(np.ascontiguousarray(np.transpose(go, (1, 2, 0))))
        xo = np.transpose(xo, (2, 0, 1))
        if flip:
            xo = xo[:, ::-1, :]
        err = elem_rel(x, xo)
        rerr = row_rel(x, xo, op.n)
        _log(f"  sub {sub} rows {R}: entry {err:.2e} row {rerr:.2e}")
        assert err <= tol and rerr <= 10 * tol


@pytest.mark.parametrize("name,nrhs", [("cfg1", 1), ("cfg1", 5), ("grf45", 2), ("even40", 3), ("wg71w16", 2),
                                       ("lens61w12", 1)])
def test_sweep_apply_parity_c128(hs, torch, name, nrhs):
    op, c = _case(name)
    _log("apply c128", name, nrhs)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C128)
    Mo = OS.factor(op, c)
    f = workloads.random_rhs(op.n, nrhs, seed=11)
    u = F.apply(torch.as_tensor(f, device="cuda")).cpu().numpy()
    uo = OS.apply_sweep(Mo, f)
    _check_apply(u, uo, op.n, TOL_C128, "c128")


@pytest.mark.parametrize("name", ["cfg1", "lens61w12"])
def test_sweep_apply_parity_c64(hs, torch, name):
    op, c = _case(name)
    _log("apply c64", name)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C64)
    Mo = OS.factor(op, c)
    f = workloads.random_rhs(op.n, 3, seed=12)
    u = F.apply(torch.as_tensor(f, device="cuda").to(torch.complex64)).cpu().numpy()
    uo = OS.apply_sweep(Mo, f.astype(np.complex64).astype(np.complex128))
    _check_apply(u.astype(np.complex128), uo, op.n, TOL_C64, "c64")


def test_gpu_preconditioner_symmetric(hs, torch):
    """x^t M y = y^t M x on the GPU path (complex symmetric LDL^t)."""
    op, c = _case("grf45")
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C128)
    x, y = workloads.random_rhs(op.n, 2, seed=21)
    My = F.apply(torch.as_tensor(y[None], device="cuda")).cpu().numpy()[0]
    Mx = F.apply(torch.as_tensor(x[None], device="cuda")).cpu().numpy()[0]
    a, b = x @ My, y @ Mx
    assert abs(a - b) <= 1e-11 * abs(a)


@pytest.mark.parametrize("prec", [0, 1])
def test_fgmres_cfg1_parity(hs, torch, prec):
    pr = workloads.cfg1()
    op = OH.Params(n=pr.n, omega=pr.omega, pml_w=pr.pml_w, mpml_w=pr.mpml_w)
    _log("fgmres cfg1 prec", prec)
    A = _gpu_problem(hs, torch, op, pr.c)
    F = hs.Factors(A, prec)
    res = hs.fgmres(A, F, torch.as_tensor(pr.f, device="cuda"), restart=20, tol=1e-6)
    u = res.u.cpu().numpy()[0]
    Ao = OH.assemble(op, pr.c)
    Mo = OS.factor(op, pr.c)
    ro = OK.fgmres(lambda v: Ao @ v, lambda v: OS.apply_sweep(Mo, v), pr.f[0], 20, 1e-6)
    true_rel = np.linalg.norm(pr.f[0] - Ao @ u) / np.linalg.norm(pr.f[0])
    err = _rel(u, ro.x)
    _log(f"  iters gpu {res.iters} oracle {ro.iters}; true relres {true_rel:.2e}; err vs oracle {err:.2e}")
    assert res.converged
    assert true_rel <= 1e-6
    assert abs(res.relres[0] - true_rel) <= 1e-9
    if prec == 0:
        assert abs(res.iters[0] - ro.iters) <= 1
        assert err <= 1e-6
    else:
        assert res.iters[0] <= ro.iters + 3
        assert err <= 1e-4


def test_fgmres_long_restart_parity(hs, torch):
    """FGMRES(30) on a case the oracle solves in 32 iterations: Arnoldi steps j >= 24 use the
    separate update and dot kernels, earlier ones the fused kernel; FP64 factors, against the
    oracle's FGMRES with the same restart and tolerance."""
    n, om = 47, 2 * math.pi * 10
    op = OH.Params(n=n, omega=om, pml_w=6, mpml_w=3)
    c = workloads.velocity_layered(n, seed=3)
    f = workloads.random_rhs(n, 1, seed=4)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C128)
    res = hs.fgmres(A, F, torch.as_tensor(f, device="cuda"), restart=30, tol=1e-11)
    Ao = OH.assemble(op, c)
    Mo = OS.factor(op, c)
    ro = OK.fgmres(lambda v: Ao @ v, lambda v: OS.apply_sweep(Mo, v), f[0], 30, 1e-11)
    u = res.u.cpu().numpy()[0]
    true_rel = np.linalg.norm(f[0] - Ao @ u) / np.linalg.norm(f[0])
    err = _rel(u, ro.x)
    _log(f"  iters gpu {res.iters} oracle {ro.iters}; true relres {true_rel:.2e}; err vs oracle {err:.2e}")
    assert ro.iters > 25
    assert res.converged and true_rel <= 1e-11
    assert abs(res.iters[0] - ro.iters) <= 1
    assert err <= 1e-8


def test_fgmres_cfg2_fp64_parity(hs, torch):
    """Config 2 (n = 255, lens, Gaussian source, widths 12) in FP64 against the oracle."""
    pr = workloads.cfg2()
    op = OH.Params(n=pr.n, omega=pr.omega, pml_w=pr.pml_w, mpml_w=pr.mpml_w)
    _log("fgmres cfg2")
    A = _gpu_problem(hs, torch, op, pr.c)
    F = hs.Factors(A, hs.HELM_C128)
    res = hs.fgmres(A, F, torch.as_tensor(pr.f, device="cuda"), restart=20, tol=1e-6)
    u = res.u.cpu().numpy()[0]
    Ao = OH.assemble(op, pr.c)
    Mo = OS.factor(op, pr.c)
    ro = OK.fgmres(lambda v: Ao @ v, lambda v: OS.apply_sweep(Mo, v), pr.f[0], 20, 1e-6)
    err = _rel(u, ro.x)
    true_rel = np.linalg.norm(pr.f[0] - Ao @ u) / np.linalg.norm(pr.f[0])
    _log(f"  iters gpu {res.iters} oracle {ro.iters}; true relres {true_rel:.2e}; err {err:.2e}")
    assert res.converged and true_rel <= 1e-6
    assert abs(res.iters[0] - ro.iters) <= 1
    assert err <= 1e-6


def test_batch_equals_individual_solves(hs, torch):
    """Uneven batch (three sizes, several right-hand sides) == per-problem solves."""
    specs = [(47, 4, 3), (63, 4, 2), (31, 4, 1)]
    probs, facs, fs, singles = [], [], [], []
    for n, w, R in specs:
        op = OH.Params(n=n, omega=2 * math.pi * n / 8, pml_w=w, mpml_w=w)
        c = workloads.velocity_layered(n, seed=n)
        A = _gpu_problem(hs, torch, op, c)
        F = hs.Factors(A, hs.HELM_C128)
        f = torch.as_tensor(workloads.random_rhs(n, R, seed=n + 1), device="cuda")
        probs.append(A); facs.append(F); fs.append(f)
        singles.append(hs.fgmres(A, F, f, restart=10, tol=1e-8))
    b = hs.Batch(probs, facs, [s[2] for s in specs], restart=10)
    res = b.solve(fs, tol=1e-8)
    assert res.converged
    k = 0
    for s, u in zip(singles, res.u):
        for q in range(len(s.iters)):
            assert res.iters[k] == s.iters[q]
            k += 1
        assert _rel(u.cpu().numpy(), s.u.cpu().numpy()) <= 1e-12


def test_error_paths_on_gpu(hs, torch):
    op, c = _case("grf45")
    c_bad = c.copy()
    c_bad[100] = float("nan")
    with pytest.raises(hs.HelmError) as ei:
        _gpu_problem(hs, torch, op, c_bad)
    assert ei.value.code == hs.HELM_EINVAL
    c_neg = c.copy()
    c_neg[7] = -1.0
    with pytest.raises(hs.HelmError):
        _gpu_problem(hs, torch, op, c_neg)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C128)
    f = torch.as_tensor(workloads.random_rhs(op.n, 1, seed=3), device="cuda")
    res = hs.fgmres(A, F, f, restart=20, tol=1e-10, maxit=1)
    assert not res.converged and res.iters == [1] and res.relres[0] > 1e-10
    with pytest.raises(hs.HelmError):
        hs.fgmres(A, F, f, tol=2.0)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_refactor_equals_individual(hs, torch, prec):
    """sweep_refactor_batch (all strips of all problems in two launches) writes the same factors as
    factoring each problem on its own: the applies agree bit for bit."""
    specs = [(47, 2), (63, 1), (39, 3)]
    probs, facs, fs, ref, cs = [], [], [], [], []
    for n, R in specs:
        op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=8, mpml_w=8)
        c = workloads.velocity_layered(n, seed=n)
        A = _gpu_problem(hs, torch, op, c)
        F = hs.Factors(A, prec)
        f = torch.as_tensor(workloads.random_rhs(n, R, seed=n + 2), device="cuda")
        if prec == hs.HELM_C64:   # complex64 factors take complex64 vectors
            f = f.to(torch.complex64)
        ref.append(F.apply(f).cpu().numpy())
        probs.append(A); facs.append(F); fs.append(f)
        cs.append(torch.as_tensor(c, dtype=torch.float64, device="cuda"))
    b = hs.Batch(probs, facs, [R for _, R in specs], restart=5)
    # leave every store holding the factors of another velocity, then restore the tables only:
    # the batched pass has to rewrite every column for the applies to match
    for A, F, c in zip(probs, facs, cs):
        A.reassemble((c * 1.25).contiguous())
        F.refactor()
        A.reassemble(c)
    b.refactor()
    for F, f, u0 in zip(facs, fs, ref):
        u = F.apply(f).cpu().numpy()
        assert np.array_equal(u, u0)


@pytest.mark.parametrize("waves", [1, 2])
@pytest.mark.parametrize("ks", [1, 2, 4])
@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_ksplit_parity(hs, torch, monkeypatch, ks, prec, waves):
    """Every right-hand-side grouping of the sweep waves (row-dot products split 1, 2 or 4 ways), with
    one or two waves per chain, gives the oracle's M f, for a single problem and for an uneven batch."""
    monkeypatch.setenv("HELM_SWEEP_SEG", "0")
    monkeypatch.setenv("HELM_SWEEP_KSPLIT", str(ks))
    monkeypatch.setenv("HELM_SWEEP_WAVES", str(waves))
    _log("ksplit", ks, "prec", prec, "waves", waves)
    op, c = _case("cfg1")
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, prec)
    Mo = OS.factor(op, c)
    f = workloads.random_rhs(op.n, 5, seed=40 + ks)
    fd = torch.as_tensor(f, device="cuda")
    if prec == hs.HELM_C64:
        u = F.apply(fd.to(torch.complex64)).cpu().numpy().astype(np.complex128)
        uo = OS.apply_sweep(Mo, f.astype(np.complex64).astype(np.complex128))
        tol = TOL_C64
    else:
        u = F.apply(fd).cpu().numpy()
        uo = OS.apply_sweep(Mo, f)
        tol = TOL_C128
    _check_apply(u, uo, op.n, tol, "single")
    # batch: this problem with 5 right-hand sides next to a smaller one with 3
    op2, c2 = _case("grf45")
    op2 = OH.Params(n=op2.n, omega=op2.omega, alpha=2.0, pml_w=8, mpml_w=8)
    A2 = _gpu_problem(hs, torch, op2, c2)
    F2 = hs.Factors(A2, prec)
    f2 = workloads.random_rhs(op2.n, 3, seed=50 + ks)
    b = hs.Batch([A, A2], [F, F2], [5, 3], restart=5)
    ub = b.apply([fd, torch.as_tensor(f2, device="cuda")])
    Mo2 = OS.factor(op2, c2)
    uo2 = OS.apply_sweep(Mo2, f2)
    # the batched apply takes complex128 vectors; with complex64 factors its error is the factors'
    btol = TOL_C128 if prec == 0 else TOL_C64
    _check_apply(ub[0].cpu().numpy(), OS.apply_sweep(Mo, f), op.n, btol, "batch 0")
    _check_apply(ub[1].cpu().numpy(), uo2, op2.n, btol, "batch 1")


def test_batch_tune_keeps_results(hs, torch):
    """The autotuner only changes the sweep schedule: after tuning, the batched application still
    gives the oracle's M f, and the chosen schedule is one of the candidates."""
    specs = [(47, 3), (63, 2), (39, 1)]
    probs, facs, fs, mos = [], [], [], []
    for n, R in specs:
        op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=8, mpml_w=8)
        c = workloads.velocity_layered(n, seed=n + 7)
        A = _gpu_problem(hs, torch, op, c)
        probs.append(A)
        facs.append(hs.Factors(A, hs.HELM_C128))
        fs.append(workloads.random_rhs(n, R, seed=n + 3))
        mos.append(OS.factor(op, c))
    b = hs.Batch(probs, facs, [R for _, R in specs], restart=4)
    choice = b.tune(reps=1)
    _log("tuned", choice)
    assert choice["ms_per_apply"] > 0
    assert choice["segmented"] == 1 or (choice["waves"] in (1, 2) and choice["ksplit"] in (1, 2, 4))
    ub = b.apply([torch.as_tensor(f, device="cuda") for f in fs])
    for u, f, Mo, (n, _) in zip(ub, fs, mos, specs):
        _check_apply(u.cpu().numpy(), OS.apply_sweep(Mo, f), n, TOL_C128, "tuned")


# (n, moving-PML width): strip heights 4, 5, 7, 9, 13; ragged last segments and exact multiples of
# the 16-column segment; a single segment (n < 16 is below the minimum size, n = 33 has three)
SEG_CASES = [(47, 3), (64, 4), (100, 6), (33, 8), (129, 8), (40, 12), (160, 12), (255, 12), (511, 12)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,w", SEG_CASES)
def test_sweep_segmented_parity(hs, torch, monkeypatch, n, w, prec):
    """The segmented chains (every strip solve split into 16-column segments joined through segment
    propagators) give the oracle's M f, alone and inside an uneven batch whose workgroups hold
    different numbers of right-hand sides."""
    monkeypatch.setenv("HELM_SWEEP_SEG", "1")
    _log("segmented", n, w, "prec", prec)
    op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=n + 17)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, prec)
    Mo = OS.factor(op, c)
    f = workloads.random_rhs(n, 3, seed=n + 5)
    fd = torch.as_tensor(f, device="cuda")
    if prec == hs.HELM_C64:
        u = F.apply(fd.to(torch.complex64)).cpu().numpy().astype(np.complex128)
        uo = OS.apply_sweep(Mo, f.astype(np.complex64).astype(np.complex128))
        tol = TOL_C64
    else:
        u = F.apply(fd).cpu().numpy()
        uo = OS.apply_sweep(Mo, f)
        tol = TOL_C128
    _check_apply(u, uo, n, tol, "single")
    # batch: next to a smaller problem of the same strip height (fewer segments, so more
    # right-hand sides per workgroup), 3 and 5 right-hand sides
    n2 = max(2 * (w + 1) + 3, n // 2 + 1)
    op2 = OH.Params(n=n2, omega=2 * math.pi * n2 / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c2 = workloads.velocity_layered(n2, seed=n2 + 3)
    A2 = _gpu_problem(hs, torch, op2, c2)
    F2 = hs.Factors(A2, prec)
    f2 = workloads.random_rhs(n2, 5, seed=n2 + 9)
    b = hs.Batch([A, A2], [F, F2], [3, 5], restart=4)
    ub = b.apply([fd, torch.as_tensor(f2, device="cuda")])
    btol = TOL_C128 if prec == 0 else TOL_C64
    _check_apply(ub[0].cpu().numpy(), OS.apply_sweep(Mo, f), n, btol, "batch 0")
    _check_apply(ub[1].cpu().numpy(), OS.apply_sweep(OS.factor(op2, c2), f2), n2, btol, "batch 1")


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_segmented_workgroup_sizes(hs, torch, monkeypatch, prec):
    """Segmented workgroups that hold several right-hand sides of a problem (the autotuner's larger
    workgroup candidates, forced through HELM_SEG_WG; complex128 halves a target beyond its 8-wave
    limit) give, bit for bit, the default grouping's M f, which matches the oracle."""
    monkeypatch.setenv("HELM_SWEEP_SEG", "1")
    specs = [(129, 8, 5), (64, 8, 3)]      # strip height 9: 9 and 4 segments, 3 and 1 waves per RHS
    probs, facs, fs, fo, mos = [], [], [], [], []
    for n, w, R in specs:
        op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
        c = workloads.velocity_layered(n, seed=n + 29)
        A = _gpu_problem(hs, torch, op, c)
        probs.append(A)
        facs.append(hs.Factors(A, prec))
        f = workloads.random_rhs(n, R, seed=n + 31)
        fo.append(f)
        fs.append(torch.as_tensor(f, device="cuda"))
        mos.append(OS.factor(op, c))
    outs = {}
    for tgt in ("0", "6", "12"):
        monkeypatch.setenv("HELM_SEG_WG", tgt)
        _log("segmented workgroup target", tgt, "prec", prec)
        b = hs.Batch(probs, facs, [R for _, _, R in specs], restart=4)
        outs[tgt] = [u.cpu().numpy() for u in b.apply(fs)]
        del b
    for tgt in ("6", "12"):
        for a, r in zip(outs[tgt], outs["0"]):
            assert np.array_equal(a, r)
    tol = TOL_C128 if prec == 0 else TOL_C64
    for u, f, Mo, (n, _, _) in zip(outs["0"], fo, mos, specs):
        _check_apply(u, OS.apply_sweep(Mo, f), n, tol, "default grouping")


def test_sweep_segmented_equals_chains(hs, torch, monkeypatch):
    """On the bench's strip height and a ragged n, a batched FGMRES solve (which freezes converged
    systems) takes the same iterations with the segmented and the plain chains, to the same answer."""
    n, w = 255, 12
    op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=5)
    f = torch.as_tensor(workloads.random_rhs(n, 4, seed=6), device="cuda")
    sols = []
    for seg in ("0", "1"):
        monkeypatch.setenv("HELM_SWEEP_SEG", seg)
        A = _gpu_problem(hs, torch, op, c)
        F = hs.Factors(A, hs.HELM_C64)
        b = hs.Batch([A], [F], [4], restart=20)
        res = b.solve([f], tol=1e-6, maxit=200)
        sols.append(res)
        _log("seg", seg, res.iters, res.relres)
    r0, r1 = sols
    assert r0.converged and r1.converged
    assert all(abs(a - c) <= 1 for a, c in zip(r0.iters, r1.iters))
    # both solutions meet the 1e-6 residual; they agree to that level times the conditioning
    assert _rel(r1.u[0].cpu().numpy(), r0.u[0].cpu().numpy()) <= 1e-4


# compressed moving chains: (n, width, segment width); ragged and whole segment counts, one segment
# (n <= 32), strip heights 4 .. 13, up to 16 segments per strip
COMP_CASES = [(47, 3, 16), (64, 4, 16), (100, 6, 32), (33, 8, 32), (129, 8, 16), (40, 12, 32), (160, 12, 32),
              (255, 12, 32), (255, 12, 16), (511, 12, 32)]


@pytest.mark.parametrize("crq", [8, 4])
@pytest.mark.parametrize("n,w,cseg", COMP_CASES)
def test_sweep_compressed_parity(hs, torch, monkeypatch, n, w, cseg, crq):
    """The compressed moving chains (every moving strip's layer-row map precomputed per segment; F / E on
    the segmented kernel) give the oracle's M f entry by entry, alone and in an uneven batch, with 8 or 4
    right-hand sides per workgroup."""
    monkeypatch.setenv("HELM_SWEEP_KIND", "2")
    monkeypatch.setenv("HELM_CSEG", str(cseg))
    monkeypatch.setenv("HELM_CRQ", str(crq))
    _log("compressed", n, w, "seg", cseg, "rq", crq)
    op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=n + 17)
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C64)
    Mo = OS.factor(op, c)
    nr = 5 if crq == 4 else 3
    f = workloads.random_rhs(n, nr, seed=n + 5)
    fd = torch.as_tensor(f, device="cuda")
    u = F.apply(fd.to(torch.complex64)).cpu().numpy().astype(np.complex128)
    uo = OS.apply_sweep(Mo, f.astype(np.complex64).astype(np.complex128))
    _check_apply(u, uo, n, TOL_C64, "single")
    n2 = max(2 * (w + 1) + 3, n // 2 + 1)
    op2 = OH.Params(n=n2, omega=2 * math.pi * n2 / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c2 = workloads.velocity_layered(n2, seed=n2 + 3)
    A2 = _gpu_problem(hs, torch, op2, c2)
    F2 = hs.Factors(A2, hs.HELM_C64)
    f2 = workloads.random_rhs(n2, 9, seed=n2 + 9)
    b = hs.Batch([A, A2], [F, F2], [nr, 9], restart=4)
    ub = b.apply([fd, torch.as_tensor(f2, device="cuda")])
    _check_apply(ub[0].cpu().numpy(), OS.apply_sweep(Mo, f), n, TOL_C64, "batch 0")
    _check_apply(ub[1].cpu().numpy(), OS.apply_sweep(OS.factor(op2, c2), f2), n2, TOL_C64, "batch 1")


def test_sweep_compressed_deterministic(hs, torch, monkeypatch):
    """Factorisation, compression and the compressed chains have no atomics and no order-dependent sums,
    so repeated factorisations and applications give the same bits: a race between the threads of
    k_compress (z, Lambda^-1 and -E/s2 are double-buffered across its steps) or between the waves of
    k_chainC (hand-off by ready flags) would show up here as differing results.  n = 511 (16 segments
    per strip, the bench's largest chains), both sweep directions of every strip parity."""
    monkeypatch.setenv("HELM_SWEEP_KIND", "2")
    monkeypatch.setenv("HELM_CSEG", "32")
    monkeypatch.setenv("HELM_CRQ", "4")
    n, w = 511, 12
    op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=23)
    A = _gpu_problem(hs, torch, op, c)
    fd = torch.as_tensor(workloads.random_rhs(n, 8, seed=29), device="cuda").to(torch.complex64)
    ref = None
    for rep in range(3):
        F = hs.Factors(A, hs.HELM_C64)
        for _ in range(2):
            u = F.apply(fd).cpu().numpy()
            if ref is None:
                ref = u
            _log(f"  factorisation {rep}: max |u - u_0| = {np.abs(u - ref).max():.3e}")
            assert np.array_equal(u, ref)
        del F


def test_sweep_compressed_fgmres(hs, torch, monkeypatch):
    """Batched FGMRES with the compressed chains takes the segmented chains' iterations (+-1) and both
    solutions meet the 1e-6 true residual."""
    n, w = 255, 12
    op = OH.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=5)
    f = torch.as_tensor(workloads.random_rhs(n, 4, seed=6), device="cuda")
    Ao = OH.assemble(op, c)
    sols = []
    for kind in ("1", "2"):
        monkeypatch.setenv("HELM_SWEEP_KIND", kind)
        A = _gpu_problem(hs, torch, op, c)
        F = hs.Factors(A, hs.HELM_C64)
        b = hs.Batch([A], [F], [4], restart=20)
        res = b.solve([f], tol=1e-6, maxit=200)
        _log("kind", kind, res.iters, res.relres)
        u = res.u[0].cpu().numpy()
        fo = f.cpu().numpy()
        rr = max(np.linalg.norm(fo[q] - Ao @ u[q]) / np.linalg.norm(fo[q]) for q in range(4))
        assert res.converged and rr <= 1e-6 * (1 + 1e-6)
        sols.append(res)
    assert all(abs(a - c) <= 1 for a, c in zip(sols[0].iters, sols[1].iters))
