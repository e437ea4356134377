"""The C-ABI's error paths and parameter conventions on the GPU (HELM_ESINGULAR, HELM_ENOMEM,
b_convention = 1, layers_d / exact_mode), through the binding."""
import math

import numpy as np
import pytest

import workloads
from parity_util import elem_rel, row_rel
from oracle import helmholtz as OH
from oracle import sweep as OS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    from paper_1007_4291_amd import helmsweep
    return helmsweep


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _problem(hs, torch, n, w, c, **kw):
    p = hs.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w, **kw)
    return hs.Problem(p, torch.as_tensor(c, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("prec", [0, 1])
def test_singular_pivot_reported(hs, torch, prec):
    """A velocity whose 1/c^2 overflows FP64 at one grid point (c = 1e-160 passes the finite, positive
    check) puts a non-finite entry into that column's diagonal block: the factorisation reports
    HELM_ESINGULAR instead of storing a broken factor, alone and in the batched refactorisation."""
    n, w = 47, 4
    c = workloads.velocity_layered(n, seed=2)
    A = _problem(hs, torch, n, w, c)
    F = hs.Factors(A, prec)
    bad = c.copy()
    bad[(n // 2) * n + n // 3] = 1e-160
    Ab = _problem(hs, torch, n, w, bad)      # assembly accepts it: finite and > 0
    with pytest.raises(hs.HelmError) as ei:
        hs.Factors(Ab, prec)
    assert ei.value.code == hs.HELM_ESINGULAR
    b = hs.Batch([A], [F], [1], restart=4)
    A.reassemble(torch.as_tensor(bad, dtype=torch.float64, device="cuda"))
    with pytest.raises(hs.HelmError) as ei:
        b.refactor()
    assert ei.value.code == hs.HELM_ESINGULAR
    assert "problem 0" in str(ei.value)


def test_size_precheck_reports_enomem(hs, torch):
    """A batch whose Krylov basis cannot fit in device memory is refused with HELM_ENOMEM by the size
    pre-check, before any allocation (and the library keeps working afterwards)."""
    n, w = 63, 4
    c = workloads.velocity_layered(n, seed=3)
    A = _problem(hs, torch, n, w, c)
    F = hs.Factors(A, hs.HELM_C64)
    # V alone: 257 blocks x 3e6 right-hand sides x n^2 x 16 bytes, far beyond 288 GB
    with pytest.raises(hs.HelmError) as ei:
        hs.Batch([A], [F], [3_000_000], restart=256)
    assert ei.value.code == hs.HELM_ENOMEM
    assert "free" in str(ei.value)
    b = hs.Batch([A], [F], [2], restart=4)
    f = torch.as_tensor(workloads.random_rhs(n, 2, seed=4), device="cuda")
    res = b.solve([f], tol=1e-6, maxit=100)
    assert res.converged


def test_unbuilt_modes_rejected(hs, torch):
    """layers_d > 1 and exact_mode are refused with HELM_EINVAL (the kernels run one row per step on
    fixed-height strips); layers_d = 0 or 1 is the one-row sweep."""
    n, w = 47, 4
    c = workloads.velocity_layered(n, seed=5)
    for kw in (dict(layers_d=12), dict(exact_mode=1)):
        with pytest.raises(hs.HelmError) as ei:
            _problem(hs, torch, n, w, c, **kw)
        assert ei.value.code == hs.HELM_EINVAL
    f = torch.as_tensor(workloads.random_rhs(n, 1, seed=6), device="cuda")
    u0 = hs.Factors(_problem(hs, torch, n, w, c, layers_d=0), hs.HELM_C128).apply(f)
    u1 = hs.Factors(_problem(hs, torch, n, w, c, layers_d=1), hs.HELM_C128).apply(f)
    assert torch.equal(u0, u1)


@pytest.mark.parametrize("prec", [0, 1])
def test_b_convention_literal(hs, torch, prec):
    """b_convention = 1 (eta = w h, B = w) on the GPU: width w + 1 in that convention is the default
    convention's width w bit for bit, and both match the oracle's M f in the literal convention."""
    n, w = 61, 8
    c = workloads.velocity_grf(n, seed=12)
    om = 2 * math.pi * 6
    p0 = hs.Params(n=n, omega=om, alpha=2.0, pml_w=w, mpml_w=w, b_convention=0)
    p1 = hs.Params(n=n, omega=om, alpha=2.0, pml_w=w + 1, mpml_w=w + 1, b_convention=1)
    cd = torch.as_tensor(c, dtype=torch.float64, device="cuda")
    F0 = hs.Factors(hs.Problem(p0, cd), prec)
    F1 = hs.Factors(hs.Problem(p1, cd), prec)
    f = workloads.random_rhs(n, 3, seed=13)
    fd = torch.as_tensor(f, device="cuda")
    if prec == hs.HELM_C64:
        fd = fd.to(torch.complex64)
    u0 = F0.apply(fd)
    u1 = F1.apply(fd)
    assert torch.equal(u0, u1)
    op = OH.Params(n=n, omega=om, alpha=2.0, pml_w=w + 1, mpml_w=w + 1, b_convention=1)
    fo = fd.cpu().numpy().astype(np.complex128)
    uo = OS.apply_sweep(OS.factor(op, c), fo)
    u = u1.cpu().numpy().astype(np.complex128)
    tol = (1e-11, 1e-10) if prec == 0 else (2e-6, 2e-5)
    e, r = elem_rel(u, uo), row_rel(u, uo, n)
    print(f"  b_convention=1 prec {prec}: entry {e:.2e} row {r:.2e}", flush=True)
    assert e <= tol[0] and r <= tol[1]
