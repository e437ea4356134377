"""Parity of the matrix-core sweep (factor precision HELM_C64_BF16X3) with the FP64 oracle.

The block products Lambda_t^{-1} [B x R] run on v_mfma_f32_16x16x32_bf16 in bf16x3 form: each FP32
operand x is carried as hi = bf16(x), lo = bf16(x - hi), |x - hi - lo| <= 2^-16 |x|, and a product is
lo*hi + hi*lo + hi*hi with FP32 accumulation, so every block product carries a relative error of about
2^-16 = 1.5e-5 where the FP32 path has 2^-24 = 6e-8.  The errors propagate through the same block
recurrences as the FP32 sweep's.  Observed: entry-wise 1.4e-5 .. 2.8e-5 for n = 61 .. 255 (about 2^-16:
the split's error, not its growth through the recurrences, dominates), row / 16-column-block-wise up to
2.6e-4 at n = 255.  tol_bf16x3 allows 1e-4 entry-wise and 1e-3 row / block-wise (4-7x over every
observation), growing as 2e-7 n and 2e-6 n past n = 500 like the FP32 path's linear growth.

Cases: strip heights B = 9, 13 and 17 (one and two 16-row tiles, partial K steps), partial and full
16-right-hand-side waves, complex64 and complex128 vectors, and the reduced waveguide problem (n = 255,
widths 16, 64 sources); FGMRES with the preconditioner reaches the 1e-6 true residual.
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
FLOOR = 1e-2


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


def tol_bf16x3(n):
    return (max(1e-4, 2e-7 * n), max(1e-3, 2e-6 * n))


def _check(u, uo, n, label):
    tol = tol_bf16x3(n)
    e, r, c = elem_rel(u, uo), row_rel(u, uo, n, FLOOR), col_seg_rel(u, uo, n, 16, FLOOR)
    _log(f"  {label} entry {e:.2e} row {r:.2e} colseg {c:.2e}")
    assert e <= tol[0], (label, e)
    assert r <= tol[1] and c <= tol[1], (label, r, c)
    return e


def _case(name):
    if name == "cfg1":                       # B = 9
        pr = workloads.cfg1()
        n, om, w, pw, c = pr.n, pr.omega, 8, 8, pr.c
    elif name == "lens61w12":                # B = 13
        n, om, w, pw = 61, 2 * math.pi * 6, 12, 12
        c = workloads.velocity_lens(n)
    elif name == "wg71w16":                  # B = 17: two 16-row tiles
        n, om, w, pw = 71, 2 * math.pi * 7, 16, 16
        c = workloads.velocity_waveguide(n, seed=5)
    else:
        raise KeyError(name)
    return OH.Params(n=n, omega=om, alpha=2.0, pml_w=pw, mpml_w=w), c


def _gpu_problem(hs, torch, op, c):
    gp = hs.Params(n=op.n, omega=op.omega, alpha=op.alpha, pml_w=op.pml_w, mpml_w=op.mpml_w, C=op.C)
    return hs.Problem(gp, torch.as_tensor(c, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("name,nrhs,vec", [("cfg1", 20, 64), ("lens61w12", 3, 64), ("wg71w16", 16, 64),
                                           ("wg71w16", 5, 128)])
def test_mfma_apply_parity(hs, torch, name, nrhs, vec):
    op, c = _case(name)
    _log("apply bf16x3", name, "B", op.B, "rhs", nrhs, "vectors", f"c{vec}")
    A = _gpu_problem(hs, torch, op, c)
    F = hs.Factors(A, hs.HELM_C64_BF16X3)
    Mo = OS.factor(op, c)
    f = workloads.random_rhs(op.n, nrhs, seed=31)
    dt = torch.complex64 if vec == 64 else torch.complex128
    fd = torch.as_tensor(f, device="cuda").to(dt)
    u = F.apply(fd).cpu().numpy().astype(np.complex128)
    uo = OS.apply_sweep(Mo, fd.cpu().numpy().astype(np.complex128))
    _check(u, uo, op.n, "bf16x3")


def test_mfma_reduced_waveguide(hs, torch):
    """n = 255, omega/2pi = 32, widths 16 (B = 17), the 64 point sources: the matrix-core apply against
    the oracle, and against the FP32 vector sweep on the same factors."""
    p = workloads.cfg5(n=255, freq=32.0)
    op = OH.Params(n=p.n, omega=p.omega, alpha=p.alpha, pml_w=p.pml_w, mpml_w=p.mpml_w)
    _log("reduced waveguide: n", p.n, "B", op.B, "rhs", p.nrhs)
    A = _gpu_problem(hs, torch, op, p.c)
    Fm = hs.Factors(A, hs.HELM_C64_BF16X3)
    Fv = hs.Factors(A, hs.HELM_C64)
    Mo = OS.factor(op, p.c)
    # the sources, and random right-hand sides (every entry nonzero)
    f = np.concatenate([p.f, workloads.random_rhs(op.n, 16, seed=33)])
    fd = torch.as_tensor(f, device="cuda").to(torch.complex64)
    um = Fm.apply(fd).cpu().numpy().astype(np.complex128)
    uv = Fv.apply(fd).cpu().numpy().astype(np.complex128)
    uo = OS.apply_sweep(Mo, fd.cpu().numpy().astype(np.complex128))
    _check(um, uo, op.n, "bf16x3 vs oracle")
    _log(f"  c64 vector path vs oracle entry {elem_rel(uv, uo):.2e}; bf16x3 vs c64 entry {elem_rel(um, uv):.2e}")


def test_mfma_fgmres_reduced_waveguide(hs, torch):
    """FGMRES(30) with the matrix-core preconditioner on the reduced waveguide problem (64 sources):
    every system reaches the 1e-6 true FP64 residual; the solutions agree with those of the FP32
    vector preconditioner to the accuracy both stop at."""
    p = workloads.cfg5(n=255, freq=32.0)
    op = OH.Params(n=p.n, omega=p.omega, alpha=p.alpha, pml_w=p.pml_w, mpml_w=p.mpml_w)
    A = _gpu_problem(hs, torch, op, p.c)
    Ao = OH.assemble(op, p.c, shifted=False)
    f = torch.as_tensor(p.f, device="cuda")
    rm = hs.fgmres(A, hs.Factors(A, hs.HELM_C64_BF16X3), f, restart=p.restart, tol=p.tol, maxit=400)
    rv = hs.fgmres(A, hs.Factors(A, hs.HELM_C64), f, restart=p.restart, tol=p.tol, maxit=400)
    um, uv = rm.u.cpu().numpy(), rv.u.cpu().numpy()
    rr = np.array([np.linalg.norm(p.f[q] - Ao @ um[q]) / np.linalg.norm(p.f[q]) for q in range(p.nrhs)])
    d = max(np.linalg.norm(um[q] - uv[q]) / np.linalg.norm(uv[q]) for q in range(p.nrhs))
    _log(f"  iters bf16x3 {min(rm.iters)}-{max(rm.iters)}, c64 {min(rv.iters)}-{max(rv.iters)}; "
         f"worst true relres {rr.max():.2e}; max rel diff of the solutions {d:.2e}")
    assert rm.converged and rr.max() <= 1e-6 * (1 + 1e-6)
    assert d <= 1e-4
