"""Element-wise comparison helpers shared by the GPU parity tests (no arithmetic of the method).

Every parity assertion compares the HIP result with the oracle's entry by entry:
  elem_rel(a, b) = max |a - b| / max |b|              over the whole output
  row_rel(a, b, n) = max over grid rows j (and right-hand sides) of
                     max_i |a - b| / max_i |b|         inside row j
so that an error confined to small-magnitude rows (PML rows, the strips' F / E rows, the last ragged
segment of the columns) cannot hide under the norm of the large rows.

Rounding errors of a sweep are absolute errors of the size of the quantities that are combined, so a
row or block whose values are far below the output's largest ones carries a larger relative error.
``floor`` bounds that: a row / block is compared relative to max(its own maximum, floor * the whole
output's maximum).  With floor = 1e-2 and a row tolerance t, a small block may differ by at most
1e-2 * t of the global maximum -- tighter than the entry-wise check wherever t < 100 * entry tolerance.
"""
import numpy as np


def elem_rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def row_rel(a, b, n: int, floor: float = 0.0) -> float:
    """Worst row-wise relative error of vectors laid out [..., n*n] row by row (rows of length n)."""
    a = np.asarray(a).reshape(-1, n)
    b = np.asarray(b).reshape(-1, n)
    den = np.maximum(np.abs(b).max(axis=1), floor * np.abs(b).max())
    num = np.abs(a - b).max(axis=1)
    ok = den > 0
    return float((num[ok] / den[ok]).max()) if ok.any() else float(num.max())


def col_seg_rel(a, b, n: int, seg: int = 16, floor: float = 0.0) -> float:
    """Worst relative error inside each block of `seg` consecutive columns of every row (the last
    block of a row is the ragged one when seg does not divide n)."""
    a = np.asarray(a).reshape(-1, n)
    b = np.asarray(b).reshape(-1, n)
    gmax = np.abs(b).max()
    worst = 0.0
    for c0 in range(0, n, seg):
        den = np.maximum(np.abs(b[:, c0:c0 + seg]).max(axis=1), floor * gmax)
        num = np.abs(a[:, c0:c0 + seg] - b[:, c0:c0 + seg]).max(axis=1)
        ok = den > 0
        if ok.any():
            worst = max(worst, float((num[ok] / den[ok]).max()))
    return worst
