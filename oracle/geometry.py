"""Element geometry and direction-independent element matrices (oracle).

For every element e the mesh map T_e(xi) = sum_m x_{e,m} v_m(xi) (eq.
elementTransformation) is a Q_r Lagrange interpolant of the control points;
its Jacobian J^e = sum_m x_{e,m} grad v_m^T (eq. Jacobian) is evaluated at a
tensor Gauss-Legendre rule, and

    M_e[m, n]    = int u_m u_n |J| dxi                      (eq. localMtMatrix
                                                              without sigma)
    K_{e,i}[m,n] = int (J^{-T} grad_xi u_m)_i u_n |J| dxi

so that the streaming block of eq. localGMatrix is G_e = -sum_i Omega_i K_{e,i}
and M_t = sigma_t M_e, M_s = sigma_s M_e for element-constant cross sections.

Rule size (reading; the paper only says Gauss-Legendre): n_q points per axis,
n_q = p + r in 2D and p + ceil(3r/2) in 3D, which integrates these polynomial
integrands exactly (|J| has degree 2r-1 (2D) / 3r-1 (3D) per variable, the
cofactor matrix 2r at most).
"""
from __future__ import annotations

import math

import numpy as np

from . import basis


def volume_points_per_axis(dim: int, r: int, p: int) -> int:
    return p + r if dim == 2 else p + int(math.ceil(1.5 * r))


def problem_control_points(prob) -> np.ndarray:
    """(E, (r+1)^dim, dim) control points of a problem: from its element list
    when the mesh is unstructured, else gathered from its lattice."""
    if getattr(prob, "elem_nodes", None) is not None:
        return np.asarray(prob.nodes, dtype=np.float64)[np.asarray(prob.elem_nodes)]
    return element_control_points(prob.lattice, prob.dim, prob.nx, prob.r)


def element_control_points(lattice: np.ndarray, dim: int, nx, r: int) -> np.ndarray:
    """(E, (r+1)^dim, dim) control points x_e gathered from the global lattice
    (the extraction operator x -> x_e of section 2)."""
    L = [r * nx[a] + 1 for a in range(dim)]
    E = int(np.prod(nx))
    e = np.arange(E)
    eidx = []
    rem = e.copy()
    for a in range(dim):
        eidx.append(rem % nx[a])
        rem = rem // nx[a]
    nloc = (r + 1) ** dim
    loc = np.arange(nloc)
    lidx = []
    rem = loc.copy()
    for a in range(dim):
        lidx.append(rem % (r + 1))
        rem = rem // (r + 1)
    flat = np.zeros((E, nloc), dtype=np.int64)
    stride = 1
    for a in range(dim):
        flat += (r * eidx[a][:, None] + lidx[a][None, :]) * stride
        stride *= L[a]
    return lattice[flat]


class ElementGeometry:
    """Jacobians and M, K_i for all elements."""

    def __init__(self, lattice, dim, nx, r, p, extra_points: int = 0, xe=None):
        """xe (E, (r+1)^dim, dim): the elements' control points when the mesh
        is given as an element list (then lattice and nx are not used)."""
        self.dim, self.nx, self.r, self.p = dim, tuple(nx), r, p
        nq = volume_points_per_axis(dim, r, p) + extra_points
        xq, wq = basis.gauss_legendre(nq)
        self.nq = nq
        geo_nodes = basis.equispaced_points(r)
        dg_nodes = basis.gll_points(p)
        Vg1, Dg1 = basis.lagrange(geo_nodes, xq)
        Vu1, Du1 = basis.lagrange(dg_nodes, xq)
        self.Vg, self.Gg = basis.tensor_values([Vg1] * dim, [Dg1] * dim)
        self.U, self.GU = basis.tensor_values([Vu1] * dim, [Du1] * dim)
        W = wq
        for _ in range(dim - 1):
            W = np.kron(wq, W)
        self.wq = W                                     # (Q,)
        # reference coordinates of the points, axis 0 fastest
        pts = np.array(np.meshgrid(*([xq] * dim), indexing="ij")).reshape(dim, -1)
        self.xi = pts[::-1].T.copy()                    # (Q, dim)
        if xe is None:
            xe = element_control_points(lattice, dim, nx, r)
        self.xe = np.asarray(xe, dtype=np.float64)               # (E, Nv, dim)
        # J[e, q, a, b] = d x_a / d xi_b
        self.J = np.einsum("ema,qmb->eqab", self.xe, self.Gg)
        self.detJ = np.linalg.det(self.J)
        self.x = np.einsum("ema,qm->eqa", self.xe, self.Vg)        # physical points

    def check_positive(self):
        mn = float(self.detJ.min())
        if not mn > 0.0:
            raise ValueError(f"non-positive Jacobian determinant {mn}")
        return mn

    def mass(self) -> np.ndarray:
        wdet = self.wq[None, :] * self.detJ                              # (E, Q)
        return np.einsum("eq,qm,qn->emn", wdet, self.U, self.U, optimize=True)

    def grad_moments(self) -> np.ndarray:
        """K[e, i, m, n] = int (d u_m / d x_i) u_n dx."""
        Jinv = np.linalg.inv(self.J)                                      # (E,Q,b,a)
        # physical gradient of u_m: (grad_x u_m)_i = sum_b Jinv[b, i] d_b u_m
        gx = np.einsum("eqbi,qmb->eqmi", Jinv, self.GU, optimize=True)
        wdet = self.wq[None, :] * self.detJ
        return np.einsum("eq,eqmi,qn->eimn", wdet, gx, self.U, optimize=True)

    def load(self, f_values: np.ndarray) -> np.ndarray:
        """int f u_m dx for f given at the physical quadrature points (E, Q)."""
        wdet = self.wq[None, :] * self.detJ
        return np.einsum("eq,eq,qm->em", wdet, f_values, self.U)

    def dg_node_positions(self) -> np.ndarray:
        """Physical positions of the DG nodes, (E, n, dim)."""
        dg_nodes = basis.gll_points(self.p)
        Vg1, _ = basis.lagrange(basis.equispaced_points(self.r), dg_nodes)
        Vn, _ = basis.tensor_values([Vg1] * self.dim, [Vg1] * self.dim)
        return np.einsum("ema,km->eka", self.xe, Vn)
