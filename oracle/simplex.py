"""Triangles and tetrahedra: the simplicial elements of section 2 (oracle).

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

Tetrahedra, the same readings one dimension up.  Reference tetrahedron with
vertices V0 = (0,0,0), V1 = (1,0,0), V2 = (0,1,0), V3 = (0,0,1); nodes of
order k on the lattice triples (i, j, l), i + j + l <= k, numbered with l
slowest, then j, then i.  A node's barycentric lattice coordinates are
c = (k - i - j - l, i, j, l); it sits at sum_v lambda_v V_v with
lambda_v = c_v / k (control points; DG nodes off the edges) or, for DG
nodes on an edge (two nonzero c_v), lambda_v = g_{c_v}, the Gauss-Lobatto
points of that edge.  For p <= 3 the DG set is vertices, Gauss-Lobatto edge
nodes and (p = 3) the centroid of each face: on every face it is the
triangle's DG set, and it is invariant under the symmetries of the
tetrahedron.  Slot s is the face opposite V_s, with its vertices listed as
(V1, V2, V3), (V0, V3, V2), (V0, V1, V3), (V0, V2, V1) for s = 0..3, so that
with the face's triangle coordinates (s, t) (first vertex at the origin,
second at s = 1, third at t = 1) the normal N = x_s x x_t points out of the
element; face node (a, b) of order k is the element node whose barycentric
coordinates are k - a - b, a, b on the face's three vertices (in that
order) and 0 on the opposite one.  Volume rule: the collapsed rule
xi = u, eta = v (1 - u), zeta = w (1 - u)(1 - v), weight
w_u w_v w_w (1 - u)^2 (1 - v), n_q = p + ceil(3r/2) points per direction,
exact for total degree 2 n_q - 3 >= 2p + 3r - 3 (the mass integrand: |J|
has degree 3 (r - 1)).
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


# ------------------------------------------------------------- tetrahedra
TET_FACES = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))   # vertices of slot s, outward order


def tet_lattice(k: int) -> np.ndarray:
    """(n, 3) lattice triples (i, j, l) of order k in node order (l slowest)."""
    return np.array([(i, j, l) for l in range(k + 1) for j in range(k + 1 - l) for i in range(k + 1 - j - l)],
                    dtype=np.int64)


def tet_index(k: int):
    """Dict lattice triple -> node number."""
    return {tuple(int(v) for v in t): m for m, t in enumerate(tet_lattice(k))}


def tet_n_nodes(k: int) -> int:
    return (k + 1) * (k + 2) * (k + 3) // 6


_V = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def _bary(L: np.ndarray, k: int) -> np.ndarray:
    """(n, 4) barycentric lattice coordinates of lattice triples."""
    return np.stack([k - L.sum(axis=1), L[:, 0], L[:, 1], L[:, 2]], axis=1)


def tet_geometry_nodes(r: int) -> np.ndarray:
    return tet_lattice(r) / float(r)


def tet_dg_nodes(p: int) -> np.ndarray:
    """DG node positions: Gauss-Lobatto on the edges, equispaced elsewhere."""
    g = basis.gll_points(p)
    C = _bary(tet_lattice(p), p)
    on_edge = (C > 0).sum(axis=1) <= 2
    lam = np.where(on_edge[:, None], g[C], C / float(p))
    return lam @ _V


def tet_slot_nodes(k: int, slot: int) -> np.ndarray:
    """Element nodes of face slot `slot`, listed in the face's triangle
    lattice order (node (a, b) of the face: coordinates k - a - b, a, b on
    the face's vertices)."""
    idx = tet_index(k)
    A, B, C = TET_FACES[slot]
    out = []
    for a, b in lattice(k):
        c = np.zeros(4, dtype=np.int64)
        c[A], c[B], c[C] = k - a - b, a, b
        out.append(idx[(int(c[1]), int(c[2]), int(c[3]))])
    return np.array(out, dtype=np.int64)


def tet_lagrange(nodes: np.ndarray, k: int, pts: np.ndarray):
    """Values V (Q, n) and gradients G (Q, n, 3) of the nodal P_k basis."""
    mono = [(a, b, c) for c in range(k + 1) for b in range(k + 1 - c) for a in range(k + 1 - b - c)]
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))

    def pw(t, e):
        return t ** e if e >= 0 else np.zeros_like(t)

    Vn = np.stack([nodes[:, 0] ** a * nodes[:, 1] ** b * nodes[:, 2] ** c for a, b, c in mono], axis=1)
    C = np.linalg.inv(Vn)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    Pm = np.stack([pw(x, a) * pw(y, b) * pw(z, c) for a, b, c in mono], axis=1)
    Px = np.stack([a * pw(x, a - 1) * pw(y, b) * pw(z, c) for a, b, c in mono], axis=1)
    Py = np.stack([b * pw(x, a) * pw(y, b - 1) * pw(z, c) for a, b, c in mono], axis=1)
    Pz = np.stack([c * pw(x, a) * pw(y, b) * pw(z, c - 1) for a, b, c in mono], axis=1)
    return Pm @ C, np.stack([Px @ C, Py @ C, Pz @ C], axis=-1)


def tet_collapsed_rule(nq: int):
    """Points (Q, 3) and weights (Q,) of the collapsed Gauss rule on the
    reference tetrahedron (u slowest)."""
    x, w = basis.gauss_legendre(nq)
    U, V, W_ = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    U, V, W_, WU, WV, WW = (a.reshape(-1) for a in (U, V, W_, WU, WV, WW))
    pts = np.stack([U, V * (1.0 - U), W_ * (1.0 - U) * (1.0 - V)], axis=1)
    return pts, WU * WV * WW * (1.0 - U) ** 2 * (1.0 - V)


class TetGeometry(ElementGeometry):
    """Jacobians, M and K_i of P_r tetrahedra with a P_p DG basis."""

    def __init__(self, xe, r: int, p: int, extra_points: int = 0):
        self.dim, self.r, self.p = 3, r, p
        self.nq = p + (3 * r + 1) // 2 + extra_points
        self.xi, self.wq = tet_collapsed_rule(self.nq)
        self.Vg, self.Gg = tet_lagrange(tet_geometry_nodes(r), r, self.xi)
        self.U, self.GU = tet_lagrange(tet_dg_nodes(p), p, self.xi)
        self.xe = np.asarray(xe, dtype=np.float64)
        self.J = np.einsum("ema,qmb->eqab", self.xe, self.Gg)
        self.detJ = np.linalg.det(self.J)
        self.x = np.einsum("ema,qm->eqa", self.xe, self.Vg)

    def dg_node_positions(self) -> np.ndarray:
        Vn, _ = tet_lagrange(tet_geometry_nodes(self.r), self.r, tet_dg_nodes(self.p))
        return np.einsum("ema,km->eka", self.xe, Vn)


def triangle_composite_rule(K: int, nq: int):
    """The reference triangle cut into K^2 congruent sub-triangles, each with
    the collapsed Gauss rule of nq x nq points: points (Q, 2), weights (Q,)."""
    x, w = collapsed_rule(nq)
    pts, wts = [], []
    for j in range(K):
        for i in range(K - j):
            # upward sub-triangle with corner (i, j) / K
            pts.append((np.array([i, j]) + x) / K)
            wts.append(w / K ** 2)
            if i + j < K - 1:
                # downward one: corners (i+1, j+1), (i, j+1), (i+1, j)
                pts.append((np.array([i + 1, j + 1]) - x) / K)
                wts.append(w / K ** 2)
    return np.concatenate(pts), np.concatenate(wts)
