"""Graph form of the batched FGMRES (a restart cycle captured once and replayed, with the convergence
bookkeeping on the device) against the eager form, through the C-ABI.

Both forms run the same kernels on the same values in the same order, and a system that leaves a
cycle is skipped by the same masks, so the solutions, iteration counts and residuals must be equal
bit for bit.  The eager form is checked against the oracle in test_gpu_parity.py.  Every solve here
takes several restart cycles (restart 5), so each call replays the graph several times, with eager
work on the same batch and host synchronisations between the calls.
"""
import math
import sys

import pytest

import workloads
from oracle import helmholtz as OH

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


def _batch(hs, torch, prec, restart=5, specs=((47, 4, 3), (63, 4, 2), (31, 4, 1))):
    probs, facs, fs = [], [], []
    for n, w, R in specs:
        op = OH.Params(n=n, omega=2 * math.pi * n / 8, pml_w=w, mpml_w=w)
        c = workloads.velocity_layered(n, seed=n + 11)
        gp = hs.Params(n=op.n, omega=op.omega, alpha=op.alpha, pml_w=op.pml_w, mpml_w=op.mpml_w, C=op.C)
        A = hs.Problem(gp, torch.as_tensor(c, dtype=torch.float64, device="cuda"))
        probs.append(A)
        facs.append(hs.Factors(A, prec))
        fs.append(torch.as_tensor(workloads.random_rhs(n, R, seed=n + 5), device="cuda"))
    b = hs.Batch(probs, facs, [R for _, _, R in specs], restart=restart)
    return b, fs, (probs, facs)


def _same(res, ref):
    assert res.converged == ref.converged
    assert res.iters == ref.iters
    assert res.relres == ref.relres
    for u, r in zip(res.u, ref.u):
        assert bool((u == r).all())


@pytest.mark.parametrize("prec,seg", [(0, "1"), (1, "1"), (1, "0")])
def test_graph_solve_equals_eager(hs, torch, monkeypatch, prec, seg):
    # seg "0": the plain chain kernels (k-split schedule) inside the captured cycle
    monkeypatch.setenv("HELM_SWEEP_SEG", seg)
    b, fs, _keep = _batch(hs, torch, prec)
    ref = b.solve(fs, tol=1e-8)
    assert ref.converged
    assert max(ref.iters) > 5                       # more than one cycle
    _log("eager iters", ref.iters)
    b.use_graph(True)
    for rep in range(3):
        _log("graph solve", prec, seg, rep)
        res = b.solve(fs, [torch.zeros_like(f) for f in fs], tol=1e-8)   # fresh output buffers
        _same(res, ref)
        b.apply(fs)                                   # eager work on the batch between the calls
        torch.cuda.synchronize()


def test_graph_solve_maxit(hs, torch):
    """Systems stopped by maxit inside a cycle: same counts, residuals and iterates."""
    b, fs, _keep = _batch(hs, torch, 1)
    ref = b.solve(fs, tol=1e-13, maxit=7)
    assert not ref.converged and max(ref.iters) == 7
    b.use_graph(True)
    _same(b.solve(fs, tol=1e-13, maxit=7), ref)
    _same(b.solve(fs, tol=1e-13, maxit=7), ref)


def test_graph_recaptured_after_tune(hs, torch):
    """The autotuner may change the sweep schedule; the next graph solve captures it anew."""
    b, fs, _keep = _batch(hs, torch, 1)
    b.use_graph(True)
    first = b.solve(fs, tol=1e-8)
    assert first.converged
    _log("tuned", b.tune(reps=1))
    b.use_graph(False)
    ref = b.solve(fs, tol=1e-8)
    b.use_graph(True)
    _same(b.solve(fs, tol=1e-8), ref)
