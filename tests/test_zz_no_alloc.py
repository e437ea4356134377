"""The allocation-free entry point sweep_apply_noalloc (static per-GPU scratch, no device
allocation) against sweep_apply on the same factors: equal bit for bit, on consecutive calls whose
second input is smaller, in both factor precisions; and refused with HELM_ENOMEM beyond its scratch."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hs():
    from paper_1007_4291_amd import helmsweep
    return helmsweep


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _factors(hs, torch, n, w, prec, seed):
    p = hs.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=w, mpml_w=w)
    c = workloads.velocity_layered(n, seed=seed)
    A = hs.Problem(p, torch.as_tensor(c, dtype=torch.float64, device="cuda"))
    return A, hs.Factors(A, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_sweep_apply(hs, torch, prec):
    # two calls in a row, the second with a smaller input (smaller problem, fewer right-hand sides)
    cases = [(255, 12, 8), (127, 12, 3)] if prec == hs.HELM_C64 else [(127, 8, 5), (47, 4, 2)]
    dt = torch.complex64 if prec == hs.HELM_C64 else torch.complex128
    kept = []
    for k, (n, w, R) in enumerate(cases):
        print(f"noalloc prec {prec} call {k}: n={n} w={w} nrhs={R}", flush=True)
        A, F = _factors(hs, torch, n, w, prec, seed=n + k)
        f = torch.as_tensor(workloads.random_rhs(n, R, seed=n + 7), device="cuda").to(dt)
        u_na = torch.full_like(f, float("nan"))
        F.apply_noalloc(f, u_na)
        u_ref = F.apply(f)
        torch.cuda.synchronize()
        assert torch.equal(u_na, u_ref), (n, R)
        assert bool(torch.isfinite(torch.view_as_real(u_na)).all())
        kept.append((A, F))
    # the first factors again after the smaller call: the scratch keeps no state between calls
    A, F = kept[0]
    n, w, R = cases[0]
    f = torch.as_tensor(workloads.random_rhs(n, R, seed=99), device="cuda").to(dt)
    u_na = torch.empty_like(f)
    F.apply_noalloc(f, u_na)
    assert torch.equal(u_na, F.apply(f))


def test_noalloc_rejects_beyond_scratch(hs, torch):
    """A call whose tables and workspaces exceed the static scratch returns HELM_ENOMEM and leaves the
    output untouched."""
    A, F = _factors(hs, torch, 511, 12, hs.HELM_C128, seed=3)
    R = 64
    f = torch.as_tensor(workloads.random_rhs(511, R, seed=4), device="cuda")
    u = torch.zeros_like(f)
    with pytest.raises(hs.HelmError) as ei:
        F.apply_noalloc(f, u)
    assert ei.value.code == hs.HELM_ENOMEM
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert not bool(u.abs().max() > 0)
