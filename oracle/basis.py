"""1D rules and Lagrange bases on the reference interval [0, 1] (oracle).

* Gauss-Legendre rules integrate the polynomial volume and face integrands
  (section 2, end: Gauss-Legendre is the usual choice for eqs.
  localGMatrix-localMsMatrix).
* The DG basis is nodal Lagrange at the Gauss-Lobatto-Legendre points
  (reading: the paper only says "Lagrangian" basis, eq. localBasis; the GLL
  set contains both end points, so a face trace involves exactly the
  (p+1)^(dim-1) nodes on that face).
* The mesh map uses Lagrange polynomials at equispaced control points
  (reading: the paper's control points x_{e,m} = T_e(xi_m), eq.
  elementTransformation, on an unspecified node set).
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gll_points(p: int) -> np.ndarray:
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = np.sort(np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c)).real)
    return 0.5 * (np.concatenate([[-1.0], inner, [1.0]]) + 1.0)


def equispaced_points(r: int) -> np.ndarray:
    return np.linspace(0.0, 1.0, r + 1)


def lagrange(nodes: np.ndarray, x: np.ndarray):
    """Values V[k, m] = l_m(x_k) and derivatives D[k, m] = l_m'(x_k)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for m in range(n):
        for j in range(n):
            if j != m:
                V[:, m] *= (x - nodes[j]) / (nodes[m] - nodes[j])
        for j in range(n):
            if j == m:
                continue
            term = np.full(len(x), 1.0 / (nodes[m] - nodes[j]))
            for k in range(n):
                if k != m and k != j:
                    term *= (x - nodes[k]) / (nodes[m] - nodes[k])
            D[:, m] += term
    return V, D


def tensor_values(V1: list, D1: list):
    """Tensor-product values and gradients.

    V1/D1: per-axis (n_pts_a, n_fun_a) arrays (axis 0 fastest in both the
    point and the function numbering).  Returns V (P, F) and G (P, F, dim)
    with G[..., a] the derivative along reference axis a.
    """
    dim = len(V1)

    def kron_axes(mats):
        out = mats[0]
        for M in mats[1:]:
            out = np.kron(M, out)   # later axes vary slower
        return out

    V = kron_axes(V1)
    G = np.stack([kron_axes([D1[b] if b == a else V1[b] for b in range(dim)])
                  for a in range(dim)], axis=-1)
    return V, G
