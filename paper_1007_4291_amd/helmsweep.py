"""Thin ctypes binding of libhelmsweep.so (C-ABI in include/helmsweep.h).

Argument marshalling only: every step of the method runs in the HIP library.  Tensors are torch
CUDA (HIP) tensors; their data pointers and the current torch stream are handed to the C-ABI.
Importing this module fails loudly if the library has not been built (``python -m
paper_1007_4291_amd.build``); there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelmsweep.so")

HELM_OK = 0
HELM_ENOTCONV = 1
HELM_EINVAL = -1
HELM_ENOMEM = -2
HELM_EHIP = -3
HELM_ESINGULAR = -4
HELM_C128 = 0
HELM_C64 = 1
HELM_C64_BF16X3 = 2      # complex64 factors, block products on the matrix cores in bf16x3 (sweep_factor only)

# every symbol the header declares
EXPORTS = ["helm_version", "helm_last_error", "helm_assemble", "helm_reassemble", "helm_problem_n", "helm_matvec",
           "sweep_factor", "sweep_refactor", "sweep_factor_bytes", "sweep_apply", "sweep_apply_noalloc", "sweep_subsolve", "sweep_num_subproblems", "sweep_subproblem_rows",
           "fgmres_solve", "helm_batch_create", "fgmres_solve_batch", "sweep_apply_batch", "sweep_refactor_batch", "helm_batch_tune", "helm_batch_set_schedule",
           "helm_batch_set_graph", "helm_free", "sweep_free",
           "helm_batch_free", "helm_timing_enable", "helm_timing_read", "helm_calib_copy"]
PHASES = ["assemble", "factor", "sweep_fwd", "sweep_mid", "sweep_bwd", "matvec", "krylov", "sweep_front"]


class HelmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"helmsweep error {code}: {msg}")
        self.code = code


class HelmParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("omega", C.c_double), ("alpha", C.c_double), ("pml_w", C.c_int32),
                ("mpml_w", C.c_int32), ("pml_C", C.c_double), ("b_convention", C.c_int32),
                ("layers_d", C.c_int32), ("exact_mode", C.c_int32)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1007_4291_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, f64 = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "helm_version": (C.c_char_p, []),
        "helm_last_error": (C.c_char_p, []),
        "helm_assemble": (C.c_int, [C.POINTER(HelmParams), vp, vp, C.POINTER(vp)]),
        "helm_reassemble": (C.c_int, [vp, vp, vp]),
        "helm_problem_n": (C.c_int, [vp]),
        "helm_matvec": (C.c_int, [vp, vp, i32, vp, i32, vp]),
        "sweep_factor": (C.c_int, [vp, i32, vp, C.POINTER(vp)]),
        "sweep_refactor": (C.c_int, [vp, vp]),
        "sweep_factor_bytes": (C.c_int64, [vp]),
        "sweep_apply": (C.c_int, [vp, vp, vp, i32, i32, vp]),
        "sweep_apply_noalloc": (C.c_int, [vp, vp, vp, i32, i32, vp]),
        "sweep_subsolve": (C.c_int, [vp, i32, vp, vp, i32, vp]),
        "sweep_num_subproblems": (C.c_int, [vp]),
        "sweep_subproblem_rows": (C.c_int, [vp, i32]),
        "fgmres_solve": (C.c_int, [vp, vp, vp, vp, i32, i32, f64, i32, C.POINTER(i32), C.POINTER(f64), vp]),
        "helm_batch_create": (C.c_int, [C.POINTER(vp), C.POINTER(vp), C.POINTER(i32), i32, i32, vp, C.POINTER(vp)]),
        "fgmres_solve_batch": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), f64, i32, C.POINTER(i32), C.POINTER(f64), vp]),
        "sweep_apply_batch": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), vp]),
        "sweep_refactor_batch": (C.c_int, [vp, vp]),
        "helm_batch_tune": (C.c_int, [vp, C.c_int32, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "helm_batch_set_graph": (C.c_int, [vp, C.c_int32]),
        "helm_batch_set_schedule": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32]),
        "helm_calib_copy": (C.c_int, [vp, vp, C.c_int64, C.c_int32, vp]),
        "helm_free": (None, [vp]),
        "sweep_free": (None, [vp]),
        "helm_batch_free": (None, [vp]),
        "helm_timing_enable": (C.c_int, [i32]),
        "helm_timing_read": (C.c_int, [C.POINTER(f64), C.POINTER(C.c_int64), i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib() -> C.CDLL:
    return _lib


def version() -> str:
    return _lib.helm_version().decode()


def _check(rc: int, allow_notconv: bool = False) -> int:
    if rc == HELM_OK or (allow_notconv and rc == HELM_ENOTCONV):
        return rc
    raise HelmError(rc, _lib.helm_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _prec_of(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return HELM_C128
    if t.dtype == torch.complex64:
        return HELM_C64
    raise TypeError(f"expected complex128 or complex64 tensor, got {t.dtype}")


def _check_vec(t, N: int, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() % N != 0:
        raise ValueError(f"{name} has {t.numel()} elements, not a multiple of N={N}")


@dataclass
class Params:
    n: int
    omega: float
    alpha: float = 2.0
    pml_w: int = 12
    mpml_w: int = 12
    C: float = 20.0
    b_convention: int = 0
    layers_d: int = 1
    exact_mode: int = 0

    def c_struct(self) -> HelmParams:
        return HelmParams(self.n, self.omega, self.alpha, self.pml_w, self.mpml_w, self.C, self.b_convention,
                          self.layers_d, self.exact_mode)

    @property
    def B(self) -> int:
        return self.mpml_w + 1 if self.b_convention == 0 else self.mpml_w


class Problem:
    """helm_problem_t: the assembled operator (a1)."""

    def __init__(self, params: Params, c, stream=None):
        torch = _torch()
        self.params = params
        self.n = params.n
        self.N = params.n * params.n
        c = c if isinstance(c, torch.Tensor) else torch.as_tensor(c)
        c = c.to(device="cuda", dtype=torch.float64).contiguous()
        if c.numel() != self.N:
            raise ValueError(f"c has {c.numel()} values, expected n*n = {self.N}")
        h = C.c_void_p()
        p = params.c_struct()
        _check(_lib.helm_assemble(C.byref(p), C.c_void_p(c.data_ptr()), C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def reassemble(self, c, stream=None):
        """Recompute the tables in place from a new velocity (a1, no allocation)."""
        torch = _torch()
        if not (isinstance(c, torch.Tensor) and c.is_cuda and c.dtype == torch.float64 and c.is_contiguous()
                and c.numel() == self.N):
            raise ValueError("c must be a contiguous float64 device tensor with n*n values")
        _check(_lib.helm_reassemble(self._h, C.c_void_p(c.data_ptr()), C.c_void_p(_stream(stream))))

    def matvec(self, x, y=None, stream=None):
        """y = A x (FP64, eq. helmd); x complex128 or complex64 [nrhs, N] or [N]."""
        torch = _torch()
        _check_vec(x, self.N, "x")
        nrhs = x.numel() // self.N
        if y is None:
            y = torch.empty(x.shape, dtype=torch.complex128, device=x.device)
        _check_vec(y, self.N, "y")
        if y.dtype != torch.complex128 or y.numel() != x.numel():
            raise ValueError("y must be complex128 with the shape of x")
        _check(_lib.helm_matvec(self._h, C.c_void_p(x.data_ptr()), _prec_of(x), C.c_void_p(y.data_ptr()), nrhs,
                                C.c_void_p(_stream(stream))))
        return y

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:     # (module globals are gone at interpreter exit)
            _lib.helm_free(h)
            self._h = None


class Factors:
    """sweep_factors_t: factored moving-PML subproblems (a2)."""

    def __init__(self, A: Problem, prec: int = HELM_C128, stream=None):
        self.A = A
        self.prec = prec
        h = C.c_void_p()
        _check(_lib.sweep_factor(A.handle, prec, C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def refactor(self, stream=None):
        """Recompute every strip factor in place (a2, no allocation)."""
        _check(_lib.sweep_refactor(self._h, C.c_void_p(_stream(stream))))

    @property
    def nbytes(self) -> int:
        return int(_lib.sweep_factor_bytes(self._h))

    @property
    def num_subproblems(self) -> int:
        return int(_lib.sweep_num_subproblems(self._h))

    def subproblem_rows(self, sub: int) -> int:
        return int(_lib.sweep_subproblem_rows(self._h, sub))

    def apply(self, f, u=None, stream=None):
        """u = M_alpha f (a3/a4); f, u complex128 or complex64 [nrhs, N]."""
        torch = _torch()
        _check_vec(f, self.A.N, "f")
        if u is None:
            u = torch.empty_like(f)
        _check_vec(u, self.A.N, "u")
        if u.dtype != f.dtype or u.numel() != f.numel():
            raise ValueError("u must match f in dtype and size")
        _check(_lib.sweep_apply(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), f.numel() // self.A.N,
                                _prec_of(f), C.c_void_p(_stream(stream))))
        return u

    def apply_noalloc(self, f, u, stream=None):
        """u = M_alpha f through the allocation-free entry point (library scratch, no device allocation);
        u must be given."""
        _check_vec(f, self.A.N, "f")
        _check_vec(u, self.A.N, "u")
        if u.dtype != f.dtype or u.numel() != f.numel():
            raise ValueError("u must match f in dtype and size")
        _check(_lib.sweep_apply_noalloc(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()),
                                        f.numel() // self.A.N, _prec_of(f), C.c_void_p(_stream(stream))))
        return u

    def subsolve(self, sub: int, g, x=None, stream=None):
        """Solve one strip with full input/output: g, x complex128 [nrhs, rows, n]."""
        torch = _torch()
        rows = self.subproblem_rows(sub)
        if rows < 0:
            raise ValueError("subproblem index out of range")
        if g.dtype != torch.complex128 or not g.is_contiguous() or g.numel() % (rows * self.A.n):
            raise ValueError("g must be contiguous complex128 [nrhs, rows, n]")
        if x is None:
            x = torch.empty_like(g)
        nrhs = g.numel() // (rows * self.A.n)
        _check(_lib.sweep_subsolve(self._h, sub, C.c_void_p(g.data_ptr()), C.c_void_p(x.data_ptr()), nrhs,
                                   C.c_void_p(_stream(stream))))
        return x

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:     # (module globals are gone at interpreter exit)
            _lib.sweep_free(h)
            self._h = None


def timing_enable(on: bool = True):
    """Record HIP events around every kernel group (per phase)."""
    _check(_lib.helm_timing_enable(1 if on else 0))


def timing_read(reset: bool = True):
    """{phase: (milliseconds, launches)} summed since the last reset."""
    ms = (C.c_double * len(PHASES))()
    ln = (C.c_int64 * len(PHASES))()
    _check(_lib.helm_timing_read(ms, ln, 1 if reset else 0))
    return {PHASES[i]: (ms[i], int(ln[i])) for i in range(len(PHASES))}


@dataclass
class SolveResult:
    u: object
    iters: List[int]
    relres: List[float]
    converged: bool


def fgmres(A: Problem, M: Factors, f, u=None, restart: int = 20, tol: float = 1e-6, maxit: int = 1000,
           stream=None) -> SolveResult:
    """Right-preconditioned FGMRES(restart) (a6); f complex128 [nrhs, N]; u = x0 in / solution out."""
    torch = _torch()
    _check_vec(f, A.N, "f")
    if f.dtype != torch.complex128:
        raise ValueError("f must be complex128")
    if u is None:
        u = torch.zeros_like(f)
    _check_vec(u, A.N, "u")
    nrhs = f.numel() // A.N
    it = (C.c_int32 * nrhs)()
    rr = (C.c_double * nrhs)()
    rc = _lib.fgmres_solve(A.handle, M.handle, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), nrhs, restart,
                           tol, maxit, it, rr, C.c_void_p(_stream(stream)))
    _check(rc, allow_notconv=True)
    return SolveResult(u, list(it), list(rr), rc == HELM_OK)


class Batch:
    """helm_batch_t: many problems of uneven size solved together (a7)."""

    def __init__(self, problems: Sequence[Problem], factors: Sequence[Factors], nrhs: Sequence[int],
                 restart: int = 20, stream=None):
        cnt = len(problems)
        self.problems, self.factors, self.nrhs = list(problems), list(factors), [int(r) for r in nrhs]
        self.restart = restart
        Ah = (C.c_void_p * cnt)(*[p.handle.value for p in problems])
        Mh = (C.c_void_p * cnt)(*[m.handle.value for m in factors])
        R = (C.c_int32 * cnt)(*self.nrhs)
        h = C.c_void_p()
        _check(_lib.helm_batch_create(Ah, Mh, R, cnt, restart, C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h

    def _ptrs(self, ts, name, dtype_ok):
        if len(ts) != len(self.problems):
            raise ValueError(f"{name}: expected {len(self.problems)} tensors")
        for t, p, r in zip(ts, self.problems, self.nrhs):
            _check_vec(t, p.N, name)
            if t.numel() != r * p.N or not dtype_ok(t):
                raise ValueError(f"{name}: wrong size or dtype")
        return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def solve(self, f: Sequence, u: Optional[Sequence] = None, tol: float = 1e-6, maxit: int = 1000, stream=None):
        torch = _torch()
        if u is None:
            u = [torch.zeros_like(t) for t in f]
        c128 = lambda t: t.dtype == torch.complex128
        fp, up = self._ptrs(f, "f", c128), self._ptrs(u, "u", c128)
        tot = sum(self.nrhs)
        it = (C.c_int32 * tot)()
        rr = (C.c_double * tot)()
        rc = _lib.fgmres_solve_batch(self._h, fp, up, tol, maxit, it, rr, C.c_void_p(_stream(stream)))
        _check(rc, allow_notconv=True)
        return SolveResult(u, list(it), list(rr), rc == HELM_OK)

    def use_graph(self, on: bool = True):
        """Run each FGMRES restart cycle of later solves as one replay of a captured hipGraph (a7)."""
        _check(_lib.helm_batch_set_graph(self._h, 1 if on else 0))

    def schedule_key(self) -> str:
        """Key of this batch's schedule in a tuning cache: strip height, factor precision and the
        multiset of (n, right-hand sides) of its members."""
        sizes = sorted((a.n, int(r)) for a, r in zip(self.problems, self.nrhs))
        runs = []
        for nr in sizes:
            if runs and runs[-1][0] == nr:
                runs[-1][1] += 1
            else:
                runs.append([nr, 1])
        p0 = self.problems[0].params
        return (f"w={p0.mpml_w};pml={p0.pml_w};bc={p0.b_convention};prec={self.factors[0].prec};"
                + ",".join(f"{c}x(n={n},R={r})" for (n, r), c in runs))

    def set_schedule(self, sched: dict):
        """Use a schedule found earlier by tune() (kind, ksplit, waves) without timing anything."""
        _check(_lib.helm_batch_set_schedule(self._h, int(sched["kind"]), int(sched["ksplit"]), int(sched["waves"])))

    def tune(self, reps: int = 2, stream=None, cache: Optional[str] = None, retune: bool = False) -> dict:
        """Pick the fastest sweep schedule for this batch by timing every candidate (a7 autotuner).

        Overwrites the batch's Krylov work space.  Returns {"kind", "segmented", "ksplit", "waves",
        "ms_per_apply"}: kind 0 plain chains (ksplit = the split, waves per chain), 1 segmented chains
        (waves = their workgroup size, ksplit 0), 2 compressed moving chains (ksplit = right-hand sides per
        workgroup, waves = its waves), 3 matrix-core chains; segmented = 1 for kinds 1 and 2.

        cache: a JSON file of schedules keyed by schedule_key().  A cached schedule is applied without
        timing (the result then has "cached": True); otherwise, or with retune, the candidates are timed
        and the winner is stored in the file."""
        import json
        key = self.schedule_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if cache and not retune and key in table:
            sched = dict(table[key])
            try:
                self.set_schedule(sched)
                sched["cached"] = True
                return sched
            except HelmError:
                pass                          # not runnable here (other library build): time again
        ks, wv, sg, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.helm_batch_tune(self._h, int(reps), C.c_void_p(_stream(stream)), C.byref(ks), C.byref(wv),
                                    C.byref(sg), C.byref(ms)))
        sched = {"kind": sg.value, "segmented": 1 if sg.value in (1, 2) else 0, "ksplit": ks.value,
                 "waves": wv.value, "ms_per_apply": ms.value}
        if cache:
            table[key] = sched
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return sched

    def refactor(self, stream=None):
        """Recompute the factors of every member in place (a2 over the whole batch, two launches)."""
        _check(_lib.sweep_refactor_batch(self._h, C.c_void_p(_stream(stream))))

    def apply(self, f: Sequence, u: Optional[Sequence] = None, stream=None):
        torch = _torch()
        if u is None:
            u = [torch.empty_like(t) for t in f]
        c128 = lambda t: t.dtype == torch.complex128
        _check(_lib.sweep_apply_batch(self._h, self._ptrs(f, "f", c128), self._ptrs(u, "u", c128),
                                      C.c_void_p(_stream(stream))))
        return u

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:     # (module globals are gone at interpreter exit)
            _lib.helm_batch_free(h)
            self._h = None


def calib_copy(src, dst, width: int, stream=None):
    """Measurement hook: copy the bytes of device tensor src into dst with width-byte (8 or 16) accesses."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size in bytes")
    _check(_lib.helm_calib_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, int(width),
                                C.c_void_p(_stream(stream))))
