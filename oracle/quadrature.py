"""Level-symmetric S_N angular quadrature (oracle).

The paper (section 2, below eq. linearSnTransport) requires positive weights
summing to 4*pi and uses level-symmetric S_2 (cosines a = sqrt(3)/3) and S_4
sets.  It prints no table, so the construction here is the textbook one:

* cosines mu_i^2 = mu_1^2 + (i-1) * 2*(1 - 3*mu_1^2)/(N-2), i = 1..N/2
  (S_2: mu_1 = 1/sqrt(3));
* octant points (mu_i, mu_j, mu_k) with i + j + k = N/2 + 2;
* one weight per permutation class, fixed by the even moment conditions
  sum_octant w * mu_x^(2m) = 1/(2m+1), m = 0..N/2-1 (least squares; the system
  is consistent: the m = 1 condition follows from mu_x^2 + mu_y^2 + mu_z^2 = 1);
* mu_1 itself is the one free parameter left, and the sets are defined by the
  next even moment, sum_octant w * mu_x^N = 1/(N+1): mu_1 is the root of that
  condition in (0, 1/sqrt(3)) at which every class weight is positive (unique
  for S_4..S_12; bracketed by a scan, refined by bisection).  The textbook
  table (S_4 0.3500212 ... S_12 0.1672126) is these roots to 7 digits;
* octant weights scaled by 4*pi/8; in 2D only the directions with a positive
  z cosine are kept and their weights doubled, so the sum stays 4*pi.

Direction order: octant o = [x<0] + 2*[y<0] (+ 4*[z<0]) ascending, then i, then
j ascending inside the octant.
"""
from __future__ import annotations

import functools
import math

import numpy as np

ORDERS = (2, 4, 6, 8, 10, 12)
# (S_16 is left out: its moment system is rank deficient, so the moment
# conditions alone do not fix its weights.)


def cosines_of(N: int, mu1: float) -> np.ndarray:
    """Level cosines mu_1 .. mu_{N/2} for a given mu_1."""
    i = np.arange(N // 2)
    return np.sqrt(mu1 ** 2 + i * 2.0 * (1.0 - 3.0 * mu1 ** 2) / (N - 2))


def _class_weights(N: int, mu: np.ndarray) -> np.ndarray:
    """Per-point octant weights (sum 1) from the moments m < N/2."""
    pts = octant_points(N)
    classes = sorted({tuple(sorted(p)) for p in pts})
    cls_of = [classes.index(tuple(sorted(p))) for p in pts]
    nm = N // 2
    A = np.zeros((nm, len(classes)))
    for m in range(nm):
        for p, c in zip(pts, cls_of):
            A[m, c] += mu[p[0]] ** (2 * m)
    b = 1.0 / (2.0 * np.arange(nm) + 1.0)
    wc, *_ = np.linalg.lstsq(A, b, rcond=None)
    return np.array([wc[c] for c in cls_of])


def next_moment_defect(N: int, mu1: float) -> float:
    """sum_octant w mu_x^N - 1/(N+1) for the set built from mu1."""
    mu = cosines_of(N, mu1)
    w = _class_weights(N, mu)
    return float(sum(wp * mu[p[0]] ** N for p, wp in zip(octant_points(N), w))) - 1.0 / (N + 1)


@functools.lru_cache(maxsize=None)
def mu1_of(N: int) -> float:
    """mu_1 of S_N: the root of the next even moment condition in
    (0, 1/sqrt(3)) with all class weights positive."""
    if N == 2:
        return 1.0 / math.sqrt(3.0)
    if N not in ORDERS:
        raise ValueError(f"no level-symmetric set for S{N}")
    grid = np.linspace(0.02, 1.0 / math.sqrt(3.0) - 1e-4, 2001)
    vals = [next_moment_defect(N, x) for x in grid]
    for k in range(len(grid) - 1):
        if vals[k] == 0.0 or vals[k] * vals[k + 1] < 0.0:
            a, b, fa = grid[k], grid[k + 1], vals[k]
            for _ in range(200):
                m = 0.5 * (a + b)
                if m <= a or m >= b:
                    break
                fm = next_moment_defect(N, m)
                if fm == 0.0:
                    a = b = m
                    break
                if (fa < 0.0) == (fm < 0.0):
                    a, fa = m, fm
                else:
                    b = m
            root = 0.5 * (a + b)
            if np.all(_class_weights(N, cosines_of(N, root)) > 0.0):
                return root
    raise ValueError(f"no positive level-symmetric set for S{N}")


def cosines(N: int) -> np.ndarray:
    if N == 2:
        return np.array([1.0 / math.sqrt(3.0)])
    return cosines_of(N, mu1_of(N))


def octant_points(N: int):
    """List of (i, j, k) index triples (0-based) in an octant, i then j."""
    h = N // 2
    pts = []
    for i in range(h):
        for j in range(h - i):
            k = h - 1 - i - j
            pts.append((i, j, k))
    return pts


def octant_weights(N: int) -> np.ndarray:
    """Octant-normalised point weights (sum 1) from the moment conditions."""
    return _class_weights(N, cosines(N))


def level_symmetric(N: int, dim: int):
    """Return (omega (D,3), w (D,)) for the level-symmetric S_N set."""
    mu = cosines(N)
    pts = octant_points(N)
    wo = octant_weights(N)
    n_oct = 8 if dim == 3 else 4
    scale = 4.0 * math.pi / 8.0 * (2.0 if dim == 2 else 1.0)
    om, ww = [], []
    for o in range(n_oct):
        sx = -1.0 if o & 1 else 1.0
        sy = -1.0 if o & 2 else 1.0
        sz = -1.0 if o & 4 else 1.0
        for (i, j, k), wp in zip(pts, wo):
            om.append((sx * mu[i], sy * mu[j], sz * mu[k]))
            ww.append(wp * scale)
    return np.array(om), np.array(ww)
