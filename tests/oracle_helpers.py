"""Independent helpers for pinning the oracle (polynomial algebra with
numpy.polynomial; no code from the oracle or the library)."""
import numpy as np
from numpy.polynomial import Polynomial as P


def lagrange_polys(nodes):
    out = []
    for m, xm in enumerate(nodes):
        poly = P([1.0])
        for j, xj in enumerate(nodes):
            if j != m:
                poly = poly * P([-xj, 1.0]) / (xm - xj)
        out.append(poly)
    return out


def gll(p):
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1
    r = np.polynomial.legendre.Legendre(c).deriv().roots().real
    return np.concatenate([[0.0], np.sort((r + 1) / 2), [1.0]])


def exact_int01(poly):
    ip = poly.integ()
    return ip(1.0) - ip(0.0)
