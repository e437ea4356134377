"""The autotuner's schedule cache (a7): a tuned schedule stored under the batch's key is applied to a
new batch of the same shape without timing, gives the same results bit for bit, and schedules a batch
cannot run are refused."""
import math
import sys

import numpy as np
import pytest

import workloads

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


def _batch(hs, torch, prec=None):
    prec = hs.HELM_C64 if prec is None else prec
    sizes = [(100, 3), (160, 2), (100, 1)]
    A, M = [], []
    for k, (n, r) in enumerate(sizes):
        c = workloads.velocity_layered(n, seed=900 + k)
        gp = hs.Params(n=n, omega=2 * math.pi * n / 8, alpha=2.0, pml_w=12, mpml_w=12)
        A.append(hs.Problem(gp, torch.as_tensor(c, dtype=torch.float64, device="cuda")))
        M.append(hs.Factors(A[-1], prec))
    return A, M, hs.Batch(A, M, [r for _, r in sizes], restart=20), sizes


def _apply(hs, torch, b, sizes, seed):
    f = [torch.as_tensor(workloads.random_rhs(n, r, seed=seed + k), device="cuda") for k, (n, r) in enumerate(sizes)]
    return [u.cpu().numpy() for u in b.apply(f)]


def test_schedule_cache_roundtrip(hs, torch, tmp_path):
    cache = str(tmp_path / "schedules.json")
    A, M, b, sizes = _batch(hs, torch)
    s1 = b.tune(reps=1, cache=cache)
    _log("tuned", s1, "key", b.schedule_key())
    assert not s1.get("cached")
    u1 = _apply(hs, torch, b, sizes, 5)
    A2, M2, b2, _ = _batch(hs, torch)
    s2 = b2.tune(reps=1, cache=cache)
    _log("cached", s2)
    assert s2.get("cached") and all(s2[k] == s1[k] for k in ("kind", "ksplit", "waves"))
    u2 = _apply(hs, torch, b2, sizes, 5)
    assert all(np.array_equal(x, y) for x, y in zip(u1, u2))
    # retune times again
    s3 = b2.tune(reps=1, cache=cache, retune=True)
    assert not s3.get("cached")


def test_schedule_refused(hs, torch):
    A, M, b, sizes = _batch(hs, torch)
    with pytest.raises(hs.HelmError):
        b.set_schedule({"kind": 3, "ksplit": 16, "waves": 1})       # needs HELM_C64_BF16X3 factors
    with pytest.raises(hs.HelmError):
        b.set_schedule({"kind": 0, "ksplit": 3, "waves": 1})        # 3 does not divide a wave's lanes
    with pytest.raises(hs.HelmError):
        b.set_schedule({"kind": 2, "ksplit": 5, "waves": 16})
    # every kind the batch offers is accepted and computes the same operator
    u = []
    for sched in ({"kind": 0, "ksplit": 1, "waves": 1}, {"kind": 1, "ksplit": 0, "waves": 2},
                  {"kind": 2, "ksplit": 4, "waves": 16}):
        try:
            b.set_schedule(sched)
        except hs.HelmError as e:
            _log("not available here:", sched, e)
            continue
        u.append(_apply(hs, torch, b, sizes, 9))
    assert len(u) >= 2
    for other in u[1:]:
        for x, y in zip(u[0], other):
            assert np.max(np.abs(x - y)) <= 1e-4 * np.max(np.abs(y))
