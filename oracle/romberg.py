"""Adaptive Romberg integration of the face integrands (oracle).

Section 2 (end) integrates the face matrices of eqs. localFDiagonalMatrix and
localFOffDiagonalMatrix, whose integrands max(+-Omega . n, 0) u_m u_n are only
piecewise smooth on faces where Omega . n changes sign, with Romberg
integration, and gives no tolerance or refinement strategy.  Reading:

* Romberg's method on [a, b]: the trapezoid sums T_k,0 with 2^k panels
  (each row adds the midpoints of the previous panels) and Richardson's
  extrapolation T_k,j = T_k,j-1 + (T_k,j-1 - T_k-1,j-1) / (4^j - 1).  The
  interval is accepted when two successive diagonal entries differ by at
  most the interval's tolerance in the max-norm over all components --
  or by at most 1e-14 times the largest component, the rounding level of
  the sums, which no halving can lower -- tested from the third row on (at
  least 5 points), for up to ``levels`` rows; otherwise it is halved and
  each half gets half the tolerance (down to ``max_depth`` halvings, after
  which the last diagonal entry is taken).  Halving concentrates the points
  at the kink, where the extrapolation does not converge on a single
  interval.
* Faces of hexahedra (two face coordinates): iterated, the outer rule over
  t of the inner integral over s, the inner tolerance a tenth of the
  outer.
"""
from __future__ import annotations

import numpy as np

LEVELS = 6
MAX_DEPTH = 30


def romberg(f, a: float, b: float, tol: float, levels: int = LEVELS, max_depth: int = MAX_DEPTH,
            _depth: int = 0) -> np.ndarray:
    """int_a^b f(s) ds for f(s (k,)) -> (k, m) values."""
    h = b - a
    ends = f(np.array([a, b], dtype=np.float64))
    rows = [[0.5 * h * (ends[0] + ends[1])]]
    for k in range(1, levels + 1):
        n_new = 1 << (k - 1)
        hk = h / (1 << k)
        s = a + hk * (2.0 * np.arange(n_new) + 1.0)
        row = [0.5 * rows[-1][0] + hk * f(s).sum(axis=0)]
        for j in range(1, k + 1):
            row.append(row[j - 1] + (row[j - 1] - rows[-1][j - 1]) / (4.0 ** j - 1.0))
        rows.append(row)
        if k >= 2 and np.abs(row[k] - rows[-2][k - 1]).max() <= max(tol, 1e-14 * np.abs(row[k]).max()):
            return row[k]
    if _depth >= max_depth:
        return rows[-1][-1]
    m = 0.5 * (a + b)
    return (romberg(f, a, m, 0.5 * tol, levels, max_depth, _depth + 1) +
            romberg(f, m, b, 0.5 * tol, levels, max_depth, _depth + 1))


def romberg_square(f, tol: float, levels: int = LEVELS) -> np.ndarray:
    """int over [0,1]^2 of f(s (k,), t scalar) -> (k, m), iterated (t outer)."""
    def outer(t):
        return np.stack([romberg(lambda s: f(s, float(tv)), 0.0, 1.0, 0.1 * tol, levels) for tv in t])
    return romberg(outer, 0.0, 1.0, tol, levels)
