"""Triangles: the simplicial elements of section 2 (oracle).

Section 2 allows simplicial elements next to the tensor-product ones: on a
triangle both the mesh map (eq. elementTransformation) and the DG basis (eq.
localBasis) are nodal Lagrange bases of P_k, the polynomials of total degree
at most k (k = r for the map, k = p for the flux).

Reference triangle T = {(xi, eta): xi, eta >= 0, xi + eta <= 1} with vertices
v0 = (0, 0), v1 = (1, 0), v2 = (0, 1).  Nodes of order k are indexed by the
lattice pairs (i, j), i, j >= 0, i + j <= k, numbered row by row:
index(i, j) = j (k + 1) - j (j - 1) / 2 + i.  Readings (the paper names no
node sets):
* control points of the map at the equispaced positions (i / k, j / k);
* DG nodes on the edges at (g_i, g_j) with g the k + 1 Gauss-Lobatto points
  of [0, 1] -- on every edge the Gauss-Lobatto points of that edge, the same
  trace nodes as the faces of the tensor elements -- and interior nodes at
  the equispaced positions (i / k, j / k), for k <= 3 only the centroid at
  k = 3 (unisolvent: a cubic vanishing at the nine edge nodes is a multiple
  of the bubble xi eta (1 - xi - eta), which is not zero there).  Both sets
  are invariant under the turns of the triangle, so an element's nodes do
  not depend on which vertex its local frame starts at.  For k <= 2 the two
  sets coincide.

Edges (element slots), each traversed counter-clockwise and parametrised by
s in [0, 1] from its first to its second vertex:
  slot 0: v0 -> v1, slot 1: v1 -> v2, slot 2: v2 -> v0,
so that for an orientation-preserving map the outward normal of every slot
is N = (t_y, -t_x) with t = dx/ds (the tangent turned clockwise).  The
face-local node b of a slot lies at s = g_b (lattice (b, 0), (k - b, b),
(0, k - b) on slots 0, 1, 2).

Volume rule (reading; the paper only says Gauss-Legendre): the collapsed
(Duffy) product rule xi = u, eta = v (1 - u), weight w_u w_v (1 - u), with
n_q = p + r Gauss points in u and v.  It integrates total degree 2 n_q - 2
exactly; the integrands of M and K have degree at most 2p + 2r - 2 (|J| has
degree 2 (r - 1), the cofactor matrix r - 1), so the element matrices are
exact.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .geometry import ElementGeometry


def lattice(k: int) -> np.ndarray:
    """(n, 2) lattice pairs (i, j) of order k in node order."""
    return np.array([(i, j) for j in range(k + 1) for i in range(k + 1 - j)], dtype=np.int64)


def index(k: int, i: int, j: int) -> int:
    return j * (k + 1) - j * (j - 1) // 2 + i


def n_nodes(k: int) -> int:
    return (k + 1) * (k + 2) // 2


def geometry_nodes(r: int) -> np.ndarray:
    """Equispaced control-point positions on the reference triangle."""
    return lattice(r) / float(r)


def dg_nodes(p: int) -> np.ndarray:
    """DG node positions: (g_i, g_j) on the edges, g the Gauss-Lobatto points
    of [0, 1]; (i / p, j / p) inside."""
    g = basis.gll_points(p)
    L = lattice(p)
    edge = (L[:, 0] == 0) | (L[:, 1] == 0) | (L.sum(axis=1) == p)
    return np.where(edge[:, None], np.stack([g[L[:, 0]], g[L[:, 1]]], axis=1), L / float(p))


def slot_nodes(k: int, slot: int) -> np.ndarray:
    """Element-local node numbers of a slot in the slot's own order."""
    out = []
    for b in range(k + 1):
        if slot == 0:
            i, j = b, 0
        elif slot == 1:
            i, j = k - b, b
        else:
            i, j = 0, k - b
        out.append(index(k, i, j))
    return np.array(out, dtype=np.int64)


def _monomials(k: int):
    return [(a, c) for c in range(k + 1) for a in range(k + 1 - c)]


def lagrange(nodes: np.ndarray, k: int, pts: np.ndarray):
    """Values V (Q, n) and gradients G (Q, n, 2) of the nodal P_k basis of
    `nodes` at `pts` (Vandermonde inverse in the monomials xi^a eta^c)."""
    mono = _monomials(k)
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    Vn = np.stack([nodes[:, 0] ** a * nodes[:, 1] ** c for a, c in mono], axis=1)
    C = np.linalg.inv(Vn)                    # column m: coefficients of basis m
    x, y = pts[:, 0], pts[:, 1]

    def pw(t, e):
        return t ** e if e >= 0 else np.zeros_like(t)

    Pm = np.stack([pw(x, a) * pw(y, c) for a, c in mono], axis=1)
    Px = np.stack([a * pw(x, a - 1) * pw(y, c) for a, c in mono], axis=1)
    Py = np.stack([c * pw(x, a) * pw(y, c - 1) for a, c in mono], axis=1)
    return Pm @ C, np.stack([Px @ C, Py @ C], axis=-1)


def collapsed_rule(nq: int):
    """Points (Q, 2) and weights (Q,) of the collapsed Gauss rule on T
    (u slowest)."""
    x, w = basis.gauss_legendre(nq)
    U, V = np.meshgrid(x, x, indexing="ij")
    WU, WV = np.meshgrid(w, w, indexing="ij")
    U, V, WU, WV = (a.reshape(-1) for a in (U, V, WU, WV))
    return np.stack([U, V * (1.0 - U)], axis=1), WU * WV * (1.0 - U)


class SimplexGeometry(ElementGeometry):
    """Jacobians, M and K_i of P_r triangles with a P_p DG basis; the matrix
    methods (mass, grad_moments, load) are those of the tensor elements."""

    def __init__(self, xe, r: int, p: int, extra_points: int = 0):
        """xe (E, (r+1)(r+2)/2, 2): control points in node order."""
        self.dim, self.r, self.p = 2, r, p
        self.nq = p + r + extra_points
        self.xi, self.wq = collapsed_rule(self.nq)
        self.Vg, self.Gg = lagrange(geometry_nodes(r), r, self.xi)
        self.U, self.GU = lagrange(dg_nodes(p), p, self.xi)
        self.xe = np.asarray(xe, dtype=np.float64)
        self.J = np.einsum("ema,qmb->eqab", self.xe, self.Gg)
        self.detJ = np.linalg.det(self.J)
        self.x = np.einsum("ema,qm->eqa", self.xe, self.Vg)

    def dg_node_positions(self) -> np.ndarray:
        Vn, _ = lagrange(geometry_nodes(self.r), self.r, dg_nodes(self.p))
        return np.einsum("ema,km->eka", self.xe, Vn)
