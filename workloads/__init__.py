"""Seeded synthetic inputs for the 2D Helmholtz sweeping-preconditioner workloads.

This module only draws velocity fields c(x) and right-hand sides f(x) on the
interior grid {(ih, jh): 1 <= i, j <= n}, h = 1/(n+1) (Section 2.1).  It holds
none of the method's arithmetic: no PML profile, no stencil, no factorisation.
Both the CPU oracle and the GPU path take their inputs from here and from
nowhere else, so the two sides see bit-identical inputs.

The paper describes its velocity fields and forces only qualitatively
(Section 3.1: a converging Gaussian lens, a vertical Gaussian waveguide, a
random field; a narrow Gaussian point source at (0.5, 0.125)).  The generators
below are seeded stand-ins with those shapes:

* ``lens``       c = (4/3)(1 - 0.5 exp(-32 |x - (1/2, 1/2)|^2))
* ``grf``        Gaussian random field, correlation length 0.05, mapped to [0.7, 1.3]
* ``layered``    K ~ U{5..10} horizontal layers, c_k ~ U[0.8, 1.5]
* ``waveguide``  (4/3)(1 - 0.5 exp(-32 (x1 - 1/2)^2)) (1 + 0.1 nu), nu a GRF
* ``const``      c = 1

Arrays are float64 / complex128, row-by-row ordering: index (j-1)*n + (i-1)
with x1 = ih the fast index (Section 2.1, the ordering of u and f).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

SEED_BASE = 20100700


def seed_for(cfg: int, problem: int = 0) -> int:
    """Seed convention: 20100700 + cfg*1000 + problem index."""
    return SEED_BASE + 1000 * int(cfg) + int(problem)


def grid(n: int) -> Tuple[np.ndarray, np.ndarray, float]:
    """Interior grid coordinates (X1[j-1, i-1] = ih, X2[j-1, i-1] = jh) and h."""
    h = 1.0 / (n + 1)
    t = h * np.arange(1, n + 1, dtype=np.float64)
    X1, X2 = np.meshgrid(t, t, indexing="xy")
    return X1, X2, h


# ----------------------------------------------------------------------------
# velocity fields (returned as (n*n,) float64, row-by-row)
# ----------------------------------------------------------------------------

def velocity_const(n: int, value: float = 1.0) -> np.ndarray:
    return np.full(n * n, float(value), dtype=np.float64)


def velocity_lens(n: int) -> np.ndarray:
    X1, X2, _ = grid(n)
    r2 = (X1 - 0.5) ** 2 + (X2 - 0.5) ** 2
    c = (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * r2))
    return c.reshape(-1)


def _grf(n: int, rng: np.random.Generator, ell: float) -> np.ndarray:
    """Smooth Gaussian random field: white noise filtered by exp(-|k|^2 ell^2 / 2)."""
    h = 1.0 / (n + 1)
    xi = rng.standard_normal((n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
    K1, K2 = np.meshgrid(k, k, indexing="xy")
    filt = np.exp(-(K1 ** 2 + K2 ** 2) * ell ** 2 / 2.0)
    g = np.real(np.fft.ifft2(np.fft.fft2(xi) * filt))
    return g


def velocity_grf(n: int, seed: int, ell: float = 0.05, lo: float = 0.7, hi: float = 1.3) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    g = _grf(n, rng, ell)
    c = lo + (hi - lo) * (g - g.min()) / (g.max() - g.min())
    return c.reshape(-1)


def velocity_layered(n: int, seed: int, kmin: int = 5, kmax: int = 10,
                     lo: float = 0.8, hi: float = 1.5) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    K = int(rng.integers(kmin, kmax + 1))
    interfaces = np.sort(rng.uniform(0.0, 1.0, K - 1))
    ck = rng.uniform(lo, hi, K)
    _, X2, _ = grid(n)
    layer = np.searchsorted(interfaces, X2[:, 0], side="right")  # per row j
    c = np.repeat(ck[layer][:, None], n, axis=1)
    return c.reshape(-1)


def velocity_waveguide(n: int, seed: int, ell: float = 0.05, amp: float = 0.1) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    nu = _grf(n, rng, ell)
    nu = nu / np.max(np.abs(nu))
    X1, _, _ = grid(n)
    c = (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * (X1 - 0.5) ** 2)) * (1.0 + amp * nu)
    return c.reshape(-1)


# ----------------------------------------------------------------------------
# right-hand sides (returned as (n*n,) complex128)
# ----------------------------------------------------------------------------

def source_point(n: int, i0: int, j0: int) -> np.ndarray:
    """Unit-mass point source delta/h^2 at grid point (i0, j0), 1-based."""
    h = 1.0 / (n + 1)
    f = np.zeros(n * n, dtype=np.complex128)
    f[(j0 - 1) * n + (i0 - 1)] = 1.0 / (h * h)
    return f


def source_point_at(n: int, x1: float, x2: float) -> np.ndarray:
    """Point source at the grid point nearest to (x1, x2)."""
    i0 = int(round(x1 * (n + 1)))
    j0 = int(round(x2 * (n + 1)))
    return source_point(n, min(max(i0, 1), n), min(max(j0, 1), n))


def source_gaussian(n: int, x1: float, x2: float, fwhm: float) -> np.ndarray:
    """Narrow Gaussian bump exp(-|x-x0|^2 / (2 s^2)), s = fwhm / (2 sqrt(2 ln 2))."""
    X1, X2, _ = grid(n)
    s = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    f = np.exp(-((X1 - x1) ** 2 + (X2 - x2) ** 2) / (2.0 * s * s))
    return f.reshape(-1).astype(np.complex128)


def random_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Dense complex Gaussian test vectors, shape (nrhs, n*n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal((nrhs, n * n)) + 1j * rng.standard_normal((nrhs, n * n)))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """One Helmholtz problem: grid size, frequency, widths, velocity and sources."""
    name: str
    n: int
    omega: float
    pml_w: int
    mpml_w: int
    c: np.ndarray                    # (n*n,) float64
    f: np.ndarray                    # (nrhs, n*n) complex128
    alpha: float = 2.0
    restart: int = 20
    tol: float = 1e-6
    meta: dict = field(default_factory=dict)

    @property
    def nrhs(self) -> int:
        return int(self.f.shape[0])

    @property
    def N(self) -> int:
        return self.n * self.n


def cfg1() -> Problem:
    """63x63, h=1/64, omega/2pi=8, c=1, widths 8, point source at (0.5, 0.25)."""
    n = 63
    return Problem("cfg1_const_n63", n, 2 * math.pi * 8, 8, 8, velocity_const(n),
                   source_point_at(n, 0.5, 0.25)[None, :])


def cfg2(n: int = 255, freq: float = 32.0) -> Problem:
    """255x255, omega/2pi=32, converging lens, widths 12, Gaussian source FWHM 1/32 at (0.5, 0.125)."""
    return Problem(f"cfg2_lens_n{n}", n, 2 * math.pi * freq, 12, 12, velocity_lens(n),
                   source_gaussian(n, 0.5, 0.125, 1.0 / 32.0)[None, :])


def cfg3(n: int = 1023, freq: float = 128.0) -> Problem:
    """1023x1023, omega/2pi=128, GRF velocity in [0.7, 1.3], widths 12, Gaussian FWHM one wavelength."""
    return Problem(f"cfg3_grf_n{n}", n, 2 * math.pi * freq, 12, 12, velocity_grf(n, seed_for(3)),
                   source_gaussian(n, 0.5, 0.125, 1.0 / freq)[None, :])


def cfg4_problem(n: int, k: int, nsrc: int = 8, width: int = 12) -> Problem:
    """One member of the uneven batch: layered velocity, omega/2pi = n/8, nsrc point sources."""
    idx = {127: 0, 255: 1, 511: 2}.get(n, 3) * 32 + k
    seed = seed_for(4, idx)
    c = velocity_layered(n, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    lo, hi = width + 2, n - width - 1
    ii = rng.integers(lo, hi + 1, nsrc)
    jj = rng.integers(lo, hi + 1, nsrc)
    f = np.stack([source_point(n, int(a), int(b)) for a, b in zip(ii, jj)])
    return Problem(f"cfg4_layered_n{n}_{k}", n, 2 * math.pi * n / 8.0, width, width, c, f)


def cfg4(per_size: int = 32, sizes=(127, 255, 511), nsrc: int = 8) -> List[Problem]:
    """96 problems (32 each of n = 127, 255, 511), 8 point sources each."""
    return [cfg4_problem(n, k, nsrc) for n in sizes for k in range(per_size)]


def cfg5(n: int = 2047, freq: float = 256.0, nsrc: int = 64, width: int = 16, pick=None) -> Problem:
    """2047x2047 waveguide, 64 point sources along x2 = 0.1, widths 16, FGMRES(30).

    ``pick`` (a slice or index list) keeps only some of the nsrc sources, at their own positions."""
    B = width + 1
    j0 = int(round(0.1 * (n + 1)))
    ii = np.rint(np.linspace(B + 1, n - B, nsrc)).astype(int)
    if pick is not None:
        ii = ii[pick]
    f = np.stack([source_point(n, int(i), j0) for i in ii])
    return Problem(f"cfg5_waveguide_n{n}", n, 2 * math.pi * freq, width, width,
                   velocity_waveguide(n, seed_for(5)), f, restart=30)
