"""Upwind DG discretisation of the S_N equations on a curved mesh (oracle).

Per direction d and element e the local system of eq. laggedSourceIteration is

  A_e = sigma_t M_e - sum_i Omega_i K_{e,i} + sum_{faces f of e} P_out(f)
  b_e = M_e (q_e + sigma_s/(4 pi) phi_e) + sum_{faces f} P_in(f) psi_up(f)

(eqs. localGMatrix, localMtMatrix, localMsMatrix, localFDiagonalMatrix,
localFOffDiagonalMatrix, qVectorDef).  P_out / P_in are the outflow / inflow
face blocks of ``faces``; psi_up is the upwind neighbour's trace, or the
constant incident flux on the domain boundary (vacuum: 0).  The diagonal face
block runs over *all* faces of the element, boundary faces included (reading:
the printed Gamma_{e,e} must include the domain boundary for the outflow
there).  The source is given per element (isotropic, per steradian); its load
vector is M_e q_e (exact for element-constant sources).
"""
from __future__ import annotations

import numpy as np

from . import quadrature
from .faces import FaceSet
from .geometry import ElementGeometry, problem_control_points
from .simplex import SimplexGeometry, TetGeometry

VACUUM, ISO_CONST, TABULATED = 0, 1, 2


class Discretization:
    """Direction-independent data of a problem plus per-direction helpers."""

    def __init__(self, prob, omega=None, w=None, source_fn=None, inflow_fn=None):
        """``source_fn(x (E,Q,dim), Omega (3,)) -> q_d`` replaces the element-
        constant source (its load is integrated with 4 extra Gauss points per
        axis); ``inflow_fn(x (...,dim), Omega) -> psi_inc`` replaces the
        constant incident flux.  Both are oracle-only test hooks."""
        self.prob = prob
        self.dim, self.nx, self.r, self.p = prob.dim, tuple(prob.nx), prob.r, prob.p
        self.unstructured = getattr(prob, "elem_nodes", None) is not None
        self.simplex = getattr(prob, "element", "tensor") == "simplex"
        self.E = len(prob.elem_nodes) if self.unstructured else int(np.prod(self.nx))
        if self.simplex:
            k = self.p
            self.n = (k + 1) * (k + 2) // 2 if self.dim == 2 else (k + 1) * (k + 2) * (k + 3) // 6
        else:
            self.n = (self.p + 1) ** self.dim
        if omega is None:
            omega, w = quadrature.level_symmetric(prob.sn_order, prob.dim)
        self.omega, self.w = np.asarray(omega), np.asarray(w)
        self.D = len(self.w)
        xe = problem_control_points(prob)
        if self.simplex:
            self.geo = (SimplexGeometry if self.dim == 2 else TetGeometry)(xe, self.r, self.p)
        else:
            self.geo = ElementGeometry(prob.lattice, self.dim, self.nx, self.r, self.p, xe=xe)
        self.geo.check_positive()
        self.M = self.geo.mass()                     # (E, n, n)
        self.K = self.geo.grad_moments()             # (E, dim, n, n)
        if self.unstructured:
            self.faces = FaceSet.from_elements(prob.nodes, prob.elem_nodes, self.dim, self.r, self.p,
                                               simplex=self.simplex)
        else:
            self.faces = FaceSet(prob.lattice, self.dim, self.nx, self.r, self.p)
        if getattr(prob, "face_rule", "exact") == "romberg":
            self.faces.romberg_tol = float(getattr(prob, "face_tol", 1e-10))
        self.sigma_t = np.asarray(prob.sigma_t, dtype=np.float64)
        self.sigma_s = np.asarray(prob.sigma_s, dtype=np.float64)
        self.q = np.asarray(prob.q, dtype=np.float64)
        self.bc_kind = prob.bc_kind
        self.psi_inc = prob.psi_inc if prob.bc_kind == ISO_CONST else 0.0
        # nodal data per direction (reading: the source and the incident
        # flux are given by their values at the DG nodes, and their loads are
        # those of the DG interpolants): q_dir (D, E, n) replaces q; the
        # tabulated inflow (D, E, n) is read at the nodes of inflow boundary
        # faces
        q_dir = getattr(prob, "q_dir", None)
        self.q_dir = None if q_dir is None else np.asarray(q_dir, dtype=np.float64).reshape(-1, self.E, self.n)
        tab = getattr(prob, "psi_inc_tab", None) if prob.bc_kind == TABULATED else None
        self.psi_tab = None if tab is None else np.asarray(tab, dtype=np.float64).reshape(-1, self.E, self.n)
        # element -> slot -> (face, side, neighbour); the element's and the
        # neighbour's DG nodes on the slot, both listed in the face's (s, t)
        # order (on a lattice the same for every element: the slot's own
        # trace nodes and those of the opposite slot)
        if not self.unstructured:
            e = np.arange(self.E)
            eidx, rem = [], e.copy()
            for a in range(self.dim):
                eidx.append(rem % self.nx[a])
                rem = rem // self.nx[a]
            self.eidx = eidx
        fs = self.faces
        self.slot_face = fs.slot_face
        self.ns = self.slot_face.shape[1]                     # slots per element (2 dim, or 3)
        self.slot_side = fs.slot_side                         # (E, ns): 0 minus, 1 plus
        self.slot_nbr = np.where(self.slot_side == 0, fs.plus[self.slot_face], fs.minus[self.slot_face])
        self.slot_trace = fs.slot_trace                       # (E, 2 dim, nf)
        self.slot_up_trace = np.zeros_like(self.slot_trace)
        for f in np.nonzero(fs.interior)[0]:
            em, ep = fs.minus[f], fs.plus[f]
            sm = int(np.nonzero(self.slot_face[em] == f)[0][0])
            sp = int(np.nonzero(self.slot_face[ep] == f)[0][0])
            self.slot_up_trace[em, sm] = self.slot_trace[ep, sp]
            self.slot_up_trace[ep, sp] = self.slot_trace[em, sm]
        # face -> slot of its minus / plus element
        self.face_slot = np.full((fs.n_faces, 2), -1, dtype=np.int64)
        for e_ in range(self.E):
            for s_ in range(self.ns):
                self.face_slot[self.slot_face[e_, s_], self.slot_side[e_, s_]] = s_
        self._cache_d = None
        self._cache = None
        self.inflow_fn = inflow_fn
        self.src_load = None
        if source_fn is not None:
            fine = ((SimplexGeometry if self.dim == 2 else TetGeometry)(xe, self.r, self.p, extra_points=4)
                    if self.simplex else
                    ElementGeometry(prob.lattice, self.dim, self.nx, self.r, self.p, extra_points=4, xe=xe))
            self.src_load = np.stack([fine.load(source_fn(fine.x, self.omega[d]))
                                      for d in range(self.D)])

    # ------------------------------------------------------------------
    def dir_index(self, d: int) -> int:
        """Row of the per-direction nodal data for direction d (the data
        covers the full quadrature; a Discretization built on a subset of
        directions maps its d back through dir_rows)."""
        return int(self.dir_rows[d]) if getattr(self, "dir_rows", None) is not None else d

    def face_blocks(self, d: int):
        """Face integrals for direction d (cached for the last direction)."""
        if self._cache_d != d:
            fn = None
            if self.inflow_fn is not None:
                om = self.omega[d]
                fn = lambda x: self.inflow_fn(x, om)
            self._cache = self.faces.integrals(self.omega[d], fn)
            self._cache_d = d
        return self._cache

    def slot_blocks(self, d: int, s: int, elems: np.ndarray):
        """(P_out, P_in) of slot s for the given elements, direction d (in
        the face's (s, t) node order)."""
        Pp, Pm, *_ = self.face_blocks(d)
        fid = self.slot_face[elems, s]
        minus = (self.slot_side[elems, s] == 0)[:, None, None]   # element is the face's minus side
        return np.where(minus, Pp[fid], Pm[fid]), np.where(minus, Pm[fid], Pp[fid])

    def local_matrix(self, d: int, elems: np.ndarray) -> np.ndarray:
        """A_e for the given elements and direction d, (k, n, n)."""
        om = self.omega[d][: self.dim]
        A = self.sigma_t[elems, None, None] * self.M[elems]
        A = A - np.einsum("i,kimn->kmn", om, self.K[elems])
        rows = np.arange(len(elems))[:, None, None]
        for s in range(self.ns):
            Pout, _ = self.slot_blocks(d, s, elems)
            tn = self.slot_trace[elems, s]
            A[rows, tn[:, :, None], tn[:, None, :]] += Pout
        return A

    def volume_source(self, phi: np.ndarray, elems: np.ndarray, d: int = 0) -> np.ndarray:
        """M_e (q_e + sigma_s/(4 pi) phi_e) for the given elements, (k, n)."""
        if self.src_load is not None:
            scat = self.sigma_s[elems, None] / (4.0 * np.pi) * phi[elems]
            return self.src_load[d][elems] + np.einsum("kmn,kn->km", self.M[elems], scat)
        if self.q_dir is not None:
            src = self.q_dir[self.dir_index(d)][elems] + self.sigma_s[elems, None] / (4.0 * np.pi) * phi[elems]
            return np.einsum("kmn,kn->km", self.M[elems], src)
        src = self.q[elems, None] + self.sigma_s[elems, None] / (4.0 * np.pi) * phi[elems]
        return np.einsum("kmn,kn->km", self.M[elems], src)

    def boundary_load(self, d: int, s: int, elems: np.ndarray):
        """Inflow load of slot s from a function-valued incident flux."""
        blocks = self.face_blocks(d)
        Lp, Lm = blocks[5], blocks[6]
        fid = self.slot_face[elems, s]
        # inflow of the minus side is where g < 0 (L_minus), of the plus side
        # where g > 0 (L_plus)
        return np.where((self.slot_side[elems, s] == 0)[:, None], Lm[fid], Lp[fid])

    def local_rhs(self, d, elems, phi, psi_kept, psi_lag, lagged_mask):
        """b_e for direction d.

        psi_kept / psi_lag: (E, n) angular flux of direction d used for kept /
        lagged upwind couplings; lagged_mask (k, ns) bool marks slots whose
        inflow edge was removed from the graph (read psi_lag)."""
        b = self.volume_source(phi, elems, d)
        rows = np.arange(len(elems))[:, None]
        for s in range(self.ns):
            _, Pin = self.slot_blocks(d, s, elems)
            tn = self.slot_trace[elems, s]
            tn_up = self.slot_up_trace[elems, s]
            nbr = self.slot_nbr[elems, s]
            interior = nbr >= 0
            up = np.zeros((len(elems), self.faces.nf))
            if np.any(interior):
                nb = np.maximum(nbr, 0)[:, None]
                src = np.where(lagged_mask[:, s][:, None], psi_lag[nb, tn_up], psi_kept[nb, tn_up])
                up = np.where(interior[:, None], src, 0.0)
            if self.psi_tab is not None:
                # tabulated incident flux at this element's own face nodes
                tab = self.psi_tab[self.dir_index(d)][elems[:, None], tn]
                up = np.where(interior[:, None], up, tab)
                b[rows, tn] += np.einsum("kab,kb->ka", Pin, up)
                continue
            if self.inflow_fn is not None:
                up = np.where(interior[:, None], up, 0.0)
                b[rows, tn] += np.einsum("kab,kb->ka", Pin, up)
                bl = self.boundary_load(d, s, elems)
                b[rows, tn] += np.where(interior[:, None], 0.0, bl)
                continue
            up = np.where(interior[:, None], up, self.psi_inc)
            b[rows, tn] += np.einsum("kab,kb->ka", Pin, up)
        return b
