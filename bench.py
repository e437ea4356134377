#!/usr/bin/env python3
"""Throughput of the moving-PML sweeping preconditioner hot path on one MI355X.

One step = one pass of the whole hot path over the workload: re-assemble every problem (a1),
re-factor every moving-PML strip (a2), then solve every right-hand side of every problem to a true
FP64 relative residual of 1e-6 with FGMRES (a3-a7: sweep forward/backward, FP64 matvec, FP64
Arnoldi), all problems batched into one set of launches per phase.  Inputs are resident in HBM when
the timed region starts.

Metric: preconditioned solves/sec, reported as RHS*N unknowns/s (right-hand sides times unknowns
per problem, per second), FP32-factor batched form vs the plain FP64 form on the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|lens255|grf1023|const63]
                       [--prec c64|c128] [--fp64-steps K64] [--graph-steps KG] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0          # MI355X dense bf16 matrix peak


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cpu-baseline-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=["batched", "lens255", "grf1023", "const63", "waveguide2047",
                                                            "waveguide255"])
    ap.add_argument("--prec", default="c64", choices=["c64", "c128", "bf16x3"],
                    help="factor precision and sweep arithmetic (bf16x3: the matrix-core block products)")
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed steps of the FP64 comparison (0: skip)")
    ap.add_argument("--graph-steps", type=int, default=1,
                    help="timed steps with each restart cycle replayed as a captured hipGraph (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-size", type=int, default=32, help="problems per size in the batched workload")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1007_4291_amd", "schedules.json"),
                    help="JSON cache of tuned sweep schedules (keyed by problem sizes, RHS counts, widths, "
                         "precision); a cached schedule is applied without timing")
    ap.add_argument("--retune", action="store_true", help="time the schedule candidates even when cached")
    return ap.parse_args()


def build_workload(name: str, per_size: int):
    import workloads as W
    if name == "batched":
        probs = W.cfg4(per_size=per_size)
        desc = (f"batched uneven: {len(probs)} problems, n in {{127,255,511}} x {per_size}, omega/2pi = n/8, "
                f"layered velocity (5-10 layers, c in [0.8,1.5]), 8 point sources each, PML and moving-PML "
                f"width 12 (B=13), FGMRES(20) to 1e-6")
    elif name == "lens255":
        probs = [W.cfg2()]
        desc = "n=255, omega/2pi=32, converging lens, Gaussian source, widths 12, FGMRES(20) to 1e-6"
    elif name == "grf1023":
        probs = [W.cfg3()]
        desc = "n=1023, omega/2pi=128, Gaussian random velocity, Gaussian source, widths 12, FGMRES(20) to 1e-6"
    elif name == "waveguide255":
        probs = [W.cfg5(n=255, freq=32.0)]
        desc = ("n=255, omega/2pi=32, waveguide velocity, 64 point sources on row 26, widths 16 (B=17), "
                "FGMRES(30) to 1e-6 (the n=2047 waveguide problem's generator at n=255)")
    elif name == "waveguide2047":
        probs = [W.cfg5()]
        desc = ("n=2047, omega/2pi=256, waveguide velocity, 64 point sources on row 205, widths 16 (B=17), "
                "FGMRES(30) to 1e-6")
    else:
        probs = [W.cfg1()]
        desc = "n=63, omega/2pi=8, c=1, point source, widths 8, FGMRES(20) to 1e-6"
    return probs, desc


class Runner:
    """Device-resident problems, factors and one batch for a given factor precision."""

    def __init__(self, hs, torch, probs, prec):
        self.hs, self.torch = hs, torch
        self.c = [torch.as_tensor(p.c, dtype=torch.float64, device="cuda") for p in probs]
        self.f = [torch.as_tensor(p.f, dtype=torch.complex128, device="cuda").contiguous() for p in probs]
        self.u = [torch.zeros_like(f) for f in self.f]
        self.A = [hs.Problem(hs.Params(n=p.n, omega=p.omega, alpha=p.alpha, pml_w=p.pml_w, mpml_w=p.mpml_w), c)
                  for p, c in zip(probs, self.c)]
        self.M = [hs.Factors(A, prec) for A in self.A]
        restart = probs[0].restart
        self.batch = hs.Batch(self.A, self.M, [p.nrhs for p in probs], restart=restart)
        self.tol = probs[0].tol
        self.last = None
        self.split = []          # (setup s, solve s) of every step: assemble + factor, then FGMRES

    def step(self):
        t0 = time.perf_counter()
        for A, c in zip(self.A, self.c):
            A.reassemble(c)
        self.batch.refactor()           # synchronises
        t1 = time.perf_counter()
        for u in self.u:
            u.zero_()
        self.last = self.batch.solve(self.f, self.u, tol=self.tol, maxit=400)   # synchronises
        self.split.append((t1 - t0, time.perf_counter() - t1))
        return self.last


def timed(runner, torch, steps, warmup):
    for _ in range(warmup):
        runner.step()
    runner.split.clear()
    runner.hs.timing_read(reset=True)
    runner.hs.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = runner.step()
        if not res.converged:
            raise RuntimeError("a system did not reach the tolerance")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    runner.hs.timing_enable(False)
    phases = runner.hs.timing_read(reset=True)
    return (t1 - t0) / steps, phases


def copy_bandwidth(torch, hs, gib=1):
    """Measured HBM bandwidth, read + write bytes / time, best of 5, GB/s: of a plain torch device copy
    ("torch"), and of the library's calibration copy (helm_calib_copy, a copy of known size) with 16-
    and with 8-byte accesses -- the kernels whose traffic counters scale the profiled counters to bytes."""
    a = torch.ones(gib * 2**27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("torch", lambda: b.copy_(a)), (16, lambda: hs.calib_copy(a, b, 16)),
                     (8, lambda: hs.calib_copy(a, b, 8))):
        best = 1e30
        for _ in range(6):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        out[name] = 2 * a.numel() * 8 / best / 1e9
    assert bool((b == a).all())
    del a, b
    torch.cuda.empty_cache()
    return out


def mfma_flops(probs, B):
    """Flops the matrix-core chains' instructions execute in one launch (one phase): per strip and
    column (both passes, 2n - 1 block products), per wave of 16 right-hand sides, 6 v_mfma_f32_16x16x32_bf16
    (three bf16 products each of the real and imaginary output) per pair of 16-row tile and 32-wide K
    step, 16 x 16 x 32 x 2 flops each -- padding of the B rows to 16-row tiles included."""
    mt = (B + 15) // 16
    fl = 0
    for p in probs:
        n = p.n
        c = (n + 1) // 2 if n % 2 else n // 2 + 1
        strips = (c - 1 - B) + (n - B - c) + 2
        waves = -(-p.nrhs // 16)
        fl += waves * strips * (2 * n - 1) * 6 * mt * mt * 16 * 16 * 32 * 2
    return fl


def sweep_bytes_flops(probs, B, fac_bytes, moving_only):
    """Algorithmic HBM bytes and flops of one sweep-chain launch (one phase of M_alpha), as the method
    defines them (whatever the kernel actually moves):

    * factor reads: every strip the launch solves is read twice per phase (the column-forward and the
      column-backward pass of its block LU solve), n columns of B(B+1)/2 packed complex entries of the
      factor precision, once per problem whatever the grouping of right-hand sides;
    * vector I/O: an application reads f and writes u, 2 N R complex values of the factor precision,
      half of it per phase;
    * flops: 2 passes x n columns x B^2 complex multiply-adds (8 flops) per strip per right-hand side.

    moving_only: the launch solves the moving layers only (the compressed chains; F and E run in their
    own launch), L strips per problem instead of L + 2.
    """
    pack = B * (B + 1) // 2
    by = fl = 0
    for p in probs:
        n, R = p.n, p.nrhs
        c = (n + 1) // 2 if n % 2 else n // 2 + 1
        L = (c - 1 - B) + (n - B - c)
        strips = L if moving_only else L + 2
        by += strips * 2 * n * pack * fac_bytes + p.N * R * fac_bytes
        fl += R * strips * 2 * n * B * B * 8
    return by, fl


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_chainC_batched96_c64_traffic.json")


def measured_traffic(workload, prec_name, kind):
    """HBM bytes per chain launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by
    the copy-kernel calibration), or None when they do not describe this workload and chain kernel or
    when the kernel sources have changed since the counters were taken."""
    import hashlib
    if workload != "batched" or prec_name != "c64" or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    if tr.get("chain_kind") != kind:
        return None
    h = hashlib.sha256()
    for f in tr.get("source_files", []):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return tr["traffic_bytes_per_launch"] if h.hexdigest() == tr.get("source_sha256") else None


def _oracle_system(task):
    """One system of the sample, in a pool worker (one thread): assemble, factor (Algorithm 3, LAPACK
    band LU per strip), FGMRES with the oracle's sweep (Algorithm 4) to the workload's tolerance.
    Returns (task, factor seconds, solve seconds, iterations, solution)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import helmholtz as OH
    from oracle import krylov as OK
    from oracle import sweep as OS
    workload, per_size, k, q = task
    p = build_workload(workload, per_size)[0][k]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        op = OH.Params(n=p.n, omega=p.omega, alpha=p.alpha, pml_w=p.pml_w, mpml_w=p.mpml_w)
        Ao = OH.assemble(op, p.c)
        Mo = OS.factor(op, p.c)
        t1 = time.perf_counter()
        r = OK.fgmres(lambda v: Ao @ v, lambda v: OS.apply_sweep(Mo, v), p.f[q], p.restart, p.tol)
        t2 = time.perf_counter()
    return task, t1 - t0, t2 - t1, r.iters, r.x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_child(workload, per_size):
    """The oracle, untuned, on a bounded sample of the workload, in a process pool on the host cores
    (run in a child process that never touches the GPU): one system (problem, right-hand side) per
    worker -- for the batched workload one problem of each size class, two right-hand sides of the
    n = 127 and n = 255 problems and one of the n = 511 problem (about 25 s of CPU work in all).
    Prints one JSON record with the timings and the solutions."""
    import multiprocessing as mp

    import numpy as np
    probs = build_workload(workload, per_size)[0]
    tasks = []
    for n in sorted(set(p.n for p in probs)):
        k = [i for i, p in enumerate(probs) if p.n == n][0]
        nq = 1 if (len(probs) > 1 and n >= 511) or len(probs) == 1 else 2
        tasks += [(workload, per_size, k, q) for q in range(min(nq, probs[k].nrhs))]
    cores = min(len(tasks), 16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(processes=cores) as pool:
        res = pool.map(_oracle_system, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    work = sum(probs[k].N for (_, _, k, _) in tasks)
    cpu_s = sum(r[1] + r[2] for r in res)
    # per-system single-core cost of each size class (factorisation once per problem, shared by its
    # right-hand sides), extrapolated to the whole workload on all host cores
    per_n = {}
    for (task, tf, ts, it, _) in res:
        p = probs[task[2]]
        d = per_n.setdefault(p.n, {"factor_s": tf, "solve_s": [], "iters": []})
        d["solve_s"].append(ts)
        d["iters"].append(it)
    t_one_core = 0.0
    for p in probs:
        d = per_n[p.n]
        t_one_core += d["factor_s"] + p.nrhs * float(np.mean(d["solve_s"]))
    ncpu = os.cpu_count() or 1
    tot = sum(p.nrhs * p.N for p in probs)
    rec = {"value": work / wall, "unit": "RHS*N unknowns/s", "cores": cores, "kind": "oracle",
           "sample": (f"{len(tasks)} systems (" + ", ".join(f"n={probs[k].n} rhs {q}" for (_, _, k, q) in tasks)
                      + f"), each assemble + factor + FGMRES({probs[0].restart}) to {probs[0].tol:g} in its own "
                      f"process (numpy/scipy FP64, 1 thread each), {cores} processes in parallel: {wall:.1f} s wall, "
                      f"{cpu_s:.1f} s CPU"),
           "host": {"cpu_count": ncpu, "model": cpu_model()},
           "per_size_single_core": {str(n): {"factor_s": round(d["factor_s"], 3),
                                             "solve_s_per_rhs": round(float(np.mean(d["solve_s"])), 3),
                                             "iters": d["iters"]} for n, d in sorted(per_n.items())},
           "extrapolated_whole_workload_all_cores": {
               "value": tot / (t_one_core / min(16, ncpu)), "cores": min(16, ncpu),
               "note": "extrapolated: per-size single-core times x the workload's systems, divided over the cores"}}
    sols = [{"k": task[2], "q": task[3], "re": np.real(x).tolist(), "im": np.imag(x).tolist()}
            for (task, _, _, _, x) in res]
    return rec, sols


def cpu_baseline(workload, per_size):
    """Run cpu_baseline_child in a fresh child process (the parent has initialised the GPU) and read its
    record and solutions back."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "cpu.json")
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", out, "--workload", workload,
               "--per-size", str(per_size)]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"cpu baseline child failed: {r.stderr[-2000:]}")
        with open(out) as fh:
            d = json.load(fh)
    return d["record"], d["solutions"]


def main():
    a = parse()
    if a.cpu_baseline_child:
        rec, sols = cpu_baseline_child(a.workload, a.per_size)
        with open(a.cpu_baseline_child, "w") as fh:
            json.dump({"record": rec, "solutions": sols}, fh)
        return 0
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        print("bench.py: only the one-GPU configuration exists (no multi-GPU path in this build)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import paper_1007_4291_amd.helmsweep as hs

    probs, desc = build_workload(a.workload, a.per_size)
    prec = {"c64": hs.HELM_C64, "c128": hs.HELM_C128, "bf16x3": hs.HELM_C64_BF16X3}[a.prec]
    B = probs[0].mpml_w + 1
    tot_unknowns = sum(p.nrhs * p.N for p in probs)
    nsys = sum(p.nrhs for p in probs)
    print(f"[bench] workload {a.workload}: {len(probs)} problems, {nsys} systems, {tot_unknowns:.3e} RHS*N",
          file=sys.stderr, flush=True)

    run = Runner(hs, torch, probs, prec)
    schedule = run.batch.tune(reps=2, cache=a.tune_cache, retune=a.retune)   # autotuned schedule (setup, not timed)
    print(f"[bench] schedule {schedule}", file=sys.stderr, flush=True)
    t_step, ph = timed(run, torch, a.steps, a.warmup)
    res = run.last
    setup_s = sorted(x[0] for x in run.split)
    solve_s = sorted(x[1] for x in run.split)
    print(f"[bench] {a.prec}: {t_step * 1e3:.1f} ms/step, iters {min(res.iters)}-{max(res.iters)}",
          file=sys.stderr, flush=True)
    value = tot_unknowns / t_step
    u_main = [u.clone() for u in run.u]

    # roofline of the dominant kernel: the sweep chain kernel (forward + backward launches); with the
    # compressed chains the moving layers' kernel, timed apart from the front strips' launches
    fac_b = 16 if prec == hs.HELM_C128 else 8
    skind = schedule.get("kind", 1 if schedule.get("segmented") else 0)
    bytes_per_launch, fl = sweep_bytes_flops(probs, B, fac_b, moving_only=(skind == 2))
    ms_f, n_f = ph["sweep_fwd"]
    ms_b, n_b = ph["sweep_bwd"]
    avg_ms = (ms_f + ms_b) / max(1, n_f + n_b)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kind = {0: "plain", 1: f"segmented-{schedule.get('waves')}w", 2: f"compressed-{schedule.get('ksplit')}rq",
            3: "matrix-core"}[skind]
    traffic = measured_traffic(a.workload, a.prec, kind)
    kname = {0: f"k_sweep{'2' if schedule.get('waves') == 2 else ''} (chains)",
             1: f"k_sweepP (segmented chains, {schedule.get('waves')}-wave workgroups)",
             2: f"k_chainC (compressed moving-layer chains, {schedule.get('ksplit')} right-hand sides and "
                f"{schedule.get('waves')} waves per workgroup)",
             3: "k_chainM (matrix-core chains, bf16x3 on v_mfma_f32_16x16x32_bf16, 16 right-hand sides per wave)"}[skind] \
        + " forward/backward launches"
    if skind == 3:
        # the matrix-core chains: MFMA work (3 bf16 products per real product) against the dense bf16 peak
        mf = mfma_flops(probs, B)
        ach = mf / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 4), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / MFMA_BF16_PEAK_TFLOPS, 6), "traffic": None, "kernel": kname,
                "avg_launch_ms": round(avg_ms, 4), "launches": n_f + n_b, "mfma_flops_per_launch": int(mf),
                "algorithmic_complex_flops_per_launch": int(fl),
                "hbm_gbs_algorithmic": round(achieved, 2)}
    else:
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": int(traffic) if traffic else None,
                "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
                "launches": n_f + n_b, "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "front_strips_ms_per_step": round(ph["sweep_front"][0] / a.steps, 3),
                "tflops": round(fl / (avg_ms * 1e-3) / 1e12, 4)}
    if skind != 3:
        roof["frac_fp32_vector"] = round(roof["tflops"] / 157.3, 5)      # of the 157.3 TFLOP/s FP32 vector peak
        roof["bytes_formula"] = ("per launch: sum over problems of (strips solved) x 2 passes x n x B(B+1)/2 x "
                                 f"{fac_b} B + N x R x {fac_b} B")
        cb = copy_bandwidth(torch, hs)
        roof["measured_copy_gbs"] = round(cb["torch"], 1)     # plain device copy (torch)
        roof["calib_copy16_gbs"] = round(cb[16], 1)           # helm_calib_copy, 16-byte accesses
        roof["calib_copy8_gbs"] = round(cb[8], 1)             # the same with 8-byte accesses
        roof["frac_of_measured_copy"] = round(achieved / cb["torch"], 5)
    else:
        roof["flops_formula"] = ("per launch: sum over chains (problem, front, 16 right-hand sides) of strips x "
                                 "(2n - 1) columns x 6 MFMA x (16-row tiles)^2 x 16 x 16 x 32 x 2")

    out = {"metric": "preconditioned solves/sec (RHS*N unknowns/s) at 1e-6 residual; FP32-batched vs FP64",
           "value": value, "unit": "RHS*N unknowns/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": a.prec, "data": "synthetic",
           "config": {"workload": desc, "problems": len(probs), "systems": nsys, "B": B,
                      "restart": probs[0].restart, "tol": probs[0].tol,
                      "factor_prec": a.prec, "krylov_prec": "f64"},
           "solves_per_s": nsys / t_step,
           "t_solve_ms_median": round(solve_s[len(solve_s) // 2] * 1e3, 2),
           "t_setup_ms_median": round(setup_s[len(setup_s) // 2] * 1e3, 2),
           "iters": {"min": min(res.iters), "max": max(res.iters), "mean": float(np.mean(res.iters))},
           "max_true_relres": max(res.relres),
           "phase_ms_per_step": {k: round(v[0] / a.steps, 3) for k, v in ph.items()},
           "sweep_schedule": schedule,
           "roofline": roof}

    if a.graph_steps > 0:
        # the same step with every FGMRES restart cycle one graph replay (captured in the warm-up step)
        run.batch.use_graph(True)
        tg, _ = timed(run, torch, a.graph_steps, 1)
        same = all(bool((u1 == u2).all()) for u1, u2 in zip(run.u, u_main)) and run.last.iters == res.iters
        run.batch.use_graph(False)
        out["graph"] = {"value": tot_unknowns / tg, "ms_per_step": tg * 1e3, "steps": a.graph_steps,
                        "equals_eager": same}
        print(f"[bench] graph form: {tg * 1e3:.1f} ms/step (equal to eager: {same})", file=sys.stderr, flush=True)

    def other_leg(key, p2, name):
        """The same steps with another factor precision: its rate and the largest relative difference of
        its solutions from the main run's."""
        r2 = Runner(hs, torch, probs, p2)
        sch2 = r2.batch.tune(reps=1, cache=a.tune_cache, retune=a.retune)
        t2, _ = timed(r2, torch, a.fp64_steps, 1 if a.warmup > 0 else 0)
        err = max(float(torch.linalg.vector_norm(u1 - u2) / torch.linalg.vector_norm(u2)) for u1, u2 in zip(u_main, r2.u))
        out[key] = {"value": tot_unknowns / t2, "ms_per_step": t2 * 1e3, "iters_max": max(r2.last.iters),
                    "sweep_schedule": sch2, "max_rel_diff_of_solutions": err}
        print(f"[bench] {name}: {t2 * 1e3:.1f} ms/step; ratio {t2 / t_step:.2f}x; diff {err:.2e}", file=sys.stderr,
              flush=True)
        del r2
        torch.cuda.empty_cache()
        return t2, err

    if a.fp64_steps > 0 and prec != hs.HELM_C128:
        del run
        torch.cuda.empty_cache()
        if prec == hs.HELM_C64_BF16X3:
            other_leg("c64_vector", hs.HELM_C64, "c64 (FP32 vector sweep)")
        try:
            t64, err = other_leg("fp64", hs.HELM_C128, "c128")
            out["speedup_vs_fp64"] = t64 / t_step
            out["max_rel_err_vs_fp64_gpu"] = err
        except RuntimeError as e:        # e.g. the FP64 Krylov basis and factors exceed the device memory
            out["fp64"] = {"skipped": str(e)[:300]}
            print(f"[bench] c128 leg skipped: {e}", file=sys.stderr, flush=True)

    if a.workload in ("waveguide2047", "waveguide255"):
        out["cpu_baseline"] = {"value": None, "kind": "oracle", "skipped": (
            "one system of this workload takes the oracle several minutes (about 2000 strip factorisations and "
            "15 FGMRES iterations of 2000 banded strip solves each), beyond the bounded sample this line allows")}
    elif not a.no_cpu_baseline:
        cb, sols = cpu_baseline(a.workload, a.per_size)
        out["cpu_baseline"] = cb
        errs = []
        for d in sols:
            x = np.asarray(d["re"]) + 1j * np.asarray(d["im"])
            u_gpu = u_main[d["k"]].cpu().numpy()[d["q"]]
            errs.append(float(np.linalg.norm(u_gpu - x) / np.linalg.norm(x)))
        out["max_rel_err_vs_oracle_sample"] = max(errs)
        print(f"[bench] cpu baseline {cb['value']:.3e} RHS*N/s on {cb['cores']} processes", file=sys.stderr, flush=True)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
