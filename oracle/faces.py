"""Faces of the structured curved mesh and the upwind face integrals (oracle).

Face numbering.  For each reference axis a, faces lie on lattice planes
P = 0..nx[a]; a face is identified by (a, P, indices of the other axes).  The
element with index P-1 along a is the face's *minus* element, the one with
index P its *plus* element (-1 on the domain boundary).  The face is
parametrised by the remaining reference axes in ascending order (s, t), and
N(s) is the area-scaled normal pointing from the minus to the plus element:
  2D  axis 0: N = (t_y, -t_x), t = dx/ds;  axis 1: N = (-t_y, t_x)
  3D  axis 0, 2: N = dx/ds x dx/dt;        axis 1: N = dx/dt x dx/ds
i.e. the cofactor of the element Jacobian applied to the face's reference
normal, so that (Omega . n) ds = (Omega . N) ds_ref.

Upwind face matrices.  With g = Omega . N, for a face and direction
  P_plus [a, b] = int max(+g, 0) phi_a phi_b ds_ref
  P_minus[a, b] = int max(-g, 0) phi_a phi_b ds_ref
where phi_a are the face traces of the GLL nodal basis.  For the minus element
P_plus is the outflow block of eq. diagonalFaceMatrixBlocks and P_minus the
inflow coupling from the plus element; for the plus element the roles swap.
Sign reading (the printed eq. offDiagonalFaceMatrixBlocks and qVectorDef carry
the opposite sign of the integration by parts): the inflow coupling enters the
*right-hand side* with a plus sign, b += P_in psi_upwind, equivalently
F_{e,e'} = -P_in on the left-hand side.

Non-smooth integrands (the paper's "re-entrant faces" where Omega . n changes
sign; it uses Romberg integration with an unstated tolerance).  Reading:
* 2D: g is a polynomial of degree r-1 in s; its roots in (0,1) split the face
  into pieces on which the integrand is a polynomial, integrated exactly with
  ceil((r+2p)/2) Gauss points per piece.
* 3D: fixed composite rule, K x K sub-squares (K = 4) with (p+r)^2 Gauss points
  each (exact on faces without a sign change).
* With ``romberg_tol`` set (the paper's choice for these integrands; see
  the ``romberg`` module), every face where Omega . N changes sign -- 2D: a
  root of g in (0,1); 3D: both signs of g at the points of the fixed
  composite rule -- is integrated instead by adaptive Romberg to the
  absolute tolerance romberg_tol * int |g| ds_ref (int |g| from the rule
  above); the other faces keep their exact Gauss rule, and so do the faces
  along the direction (dropped below).
* Interior faces: a side whose inflow measure int max(-/+g, 0) ds_ref is at
  most tau = 1e-12 times int |g| ds_ref is dropped entirely (its P is set to
  zero), so the operator and the dependency graph agree; a face along the
  direction (int |g| ds_ref at most tau |int N ds_ref|, i.e. Omega . N is
  zero up to rounding) has both sides dropped.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis
from . import simplex as simplex_ref
from .romberg import romberg, romberg_square

TAU = 1e-12


class _Poly1D:
    """Lagrange polynomials of a node set as monomial coefficients (inverse
    Vandermonde), for many evaluations: val(x) (k, n), der(x) (k, n)."""

    def __init__(self, nodes):
        nodes = np.asarray(nodes, dtype=np.float64)
        self.n = len(nodes)
        self.C = np.linalg.inv(np.vander(nodes, self.n, increasing=True))
        self.dC = self.C[1:] * np.arange(1, self.n)[:, None]

    def val(self, x):
        return np.vander(x, self.n, increasing=True) @ self.C

    def der(self, x):
        return np.vander(x, self.n - 1, increasing=True) @ self.dC
KINK_SUBDIV_3D = 4


def face_rule_2d(r: int, p: int) -> int:
    return int(math.ceil((r + 2 * p) / 2.0))


class FaceSet:
    def __init__(self, lattice, dim, nx, r, p):
        self.dim, self.nx, self.r, self.p = dim, tuple(nx), r, p
        L = [r * nx[a] + 1 for a in range(dim)]
        axis, minus, plus, ctrl, idx_all = [], [], [], [], []
        self.axis_offset = []
        off = 0
        for a in range(dim):
            self.axis_offset.append(off)
            ext = [nx[b] + (1 if b == a else 0) for b in range(dim)]
            nf_a = int(np.prod(ext))
            fid = np.arange(nf_a)
            idx = []
            rem = fid.copy()
            for b in range(dim):
                idx.append(rem % ext[b])
                rem = rem // ext[b]
            P = idx[a]
            # element linear index helper
            def elem(ii):
                e = np.zeros_like(ii[0])
                s = 1
                for b in range(dim):
                    e = e + ii[b] * s
                    s *= nx[b]
                return e
            im = list(idx)
            im[a] = P - 1
            ip = list(idx)
            mi = np.where(P >= 1, elem(im), -1)
            pl = np.where(P < nx[a], elem(ip), -1)
            # face control points, remaining axes ascending, first fastest
            others = [b for b in range(dim) if b != a]
            nloc = (r + 1) ** (dim - 1)
            loc = np.arange(nloc)
            lidx = []
            rem = loc.copy()
            for _ in others:
                lidx.append(rem % (r + 1))
                rem = rem // (r + 1)
            flat = np.zeros((nf_a, nloc), dtype=np.int64)
            stride = 1
            for b in range(dim):
                if b == a:
                    coord = (r * P)[:, None] + 0 * loc[None, :]
                else:
                    k = others.index(b)
                    coord = (r * idx[b])[:, None] + lidx[k][None, :]
                flat += coord * stride
                stride *= L[b]
            axis.append(np.full(nf_a, a))
            minus.append(mi)
            plus.append(pl)
            ctrl.append(lattice[flat])
            off += nf_a
        self.axis = np.concatenate(axis)
        self.minus = np.concatenate(minus)
        self.plus = np.concatenate(plus)
        self.ctrl = np.concatenate(ctrl)          # (F, (r+1)^(dim-1), dim)
        self._finish()
        # per element slot: face, side and the element's DG nodes in the
        # face's (s, t) order (the same for every element of a lattice)
        E = int(np.prod(nx))
        e = np.arange(E)
        eidx, rem = [], e.copy()
        for a in range(dim):
            eidx.append(rem % nx[a])
            rem = rem // nx[a]
        ns = 2 * dim
        self.slot_face = np.zeros((E, ns), dtype=np.int64)
        self.slot_side = np.zeros((E, ns), dtype=np.int64)
        self.slot_trace = np.zeros((E, ns, self.nf), dtype=np.int64)
        for sl in range(ns):
            fid, side = self.face_of_slot(eidx, sl)
            self.slot_face[:, sl] = fid
            self.slot_side[:, sl] = side
            self.slot_trace[:, sl, :] = self.trace_nodes(sl)[None, :]

    romberg_tol = None   # relative tolerance of adaptive Romberg on sign-changing faces, or None

    tri_faces = False   # faces are triangles (tetrahedra)

    def _finish(self):
        self.n_faces = len(self.axis)
        self.interior = (self.minus >= 0) & (self.plus >= 0)
        if self.tri_faces:
            self.nf = (self.p + 1) * (self.p + 2) // 2
        else:
            self.nf = (self.p + 1) ** (self.dim - 1)
        self._geo_nodes = basis.equispaced_points(self.r)
        self._dg_nodes = basis.gll_points(self.p)
        if self.tri_faces:
            self._setup_tri_rule()
        elif self.dim == 3:
            self._setup_3d_rule()
        # |int N ds_ref| per face (the face's area scale)
        if self.dim == 2:
            xg, wg = basis.gauss_legendre(face_rule_2d(self.r, self.p))
            Nq = self._normals(xg[:, None], per_face=False)               # (F, Q, 2)
            self.n_area = np.linalg.norm(np.einsum("q,fqa->fa", wg, Nq), axis=1)
        else:
            self.n_area = np.linalg.norm(np.einsum("q,fqa->fa", self.rule3_w, self.rule3_N), axis=1)

    # ------------------------------------------------------------------
    @classmethod
    def from_elements(cls, nodes, elem_nodes, dim: int, r: int, p: int, simplex: bool = False):
        """Faces of a conforming mesh given as element control-point lists.

        simplex: the elements are P_r triangles (``simplex`` module: three
        counter-clockwise edge slots, whose N of the 2D axis-0 formula is the
        outward normal, so no slot is mirrored and every face has axis 0) or,
        in 3D, tetrahedra (``from_tets``).

        Two element slots are the same face when their corner control points
        coincide (by index).  Convention for each face: its minus element is
        the one with the smaller index (the only one on the boundary); the
        face is parametrised like the minus element's slot (remaining axes
        ascending), mirrored when that slot is a xi_a = 0 face (2D: s ->
        1 - s; 3D: s and t exchanged), so that N, computed from the axis
        formula above, is the outward normal of the minus element.  The plus
        element's face coordinates are related to the face's by one of the
        symmetries of the reference face, read off the positions of the
        shared control points.  Slot tables: per (element, slot) the face,
        the side (0 minus, 1 plus) and the element's DG nodes listed in the
        face's (s, t) order."""
        if simplex and dim == 3:
            return cls.from_tets(nodes, elem_nodes, r, p)
        fs = cls.__new__(cls)
        nodes = np.asarray(nodes, dtype=np.float64)
        en = np.asarray(elem_nodes, dtype=np.int64)
        E, ns = len(en), (3 if simplex else 2 * dim)
        fs.dim, fs.r, fs.p, fs.nx = dim, r, p, (E,) + (1,) * (dim - 1)
        nfc = (r + 1) ** (dim - 1)

        def face_grid(order, slot):
            """Element-local node numbers of a slot at per-axis order
            `order`, as a (order+1)^(dim-1) grid in the slot's own (s, t)."""
            a, hi = slot // 2, slot % 2
            others = [b for b in range(dim) if b != a]
            n1 = order + 1
            out = np.zeros((n1,) * (dim - 1), dtype=np.int64)
            for loc in np.ndindex(*((n1,) * (dim - 1))):
                idx = [0] * dim
                for k, b in enumerate(others):
                    idx[b] = loc[::-1][k] if dim == 3 else loc[k]
                idx[a] = order if hi else 0
                out[loc] = sum(idx[b] * n1 ** b for b in range(dim))
            return out   # 2D: out[i]; 3D: out[j, i] (t slow, s fast)

        if simplex:
            ctrl_grid = [simplex_ref.slot_nodes(r, sl) for sl in range(ns)]
            dg_grid = [simplex_ref.slot_nodes(p, sl) for sl in range(ns)]
        else:
            ctrl_grid = [face_grid(r, sl) for sl in range(ns)]
            dg_grid = [face_grid(p, sl) for sl in range(ns)]

        def corners(g):
            return (g[0], g[-1]) if dim == 2 else (g[0, 0], g[0, -1], g[-1, 0], g[-1, -1])

        table = {}
        for e in range(E):
            for sl in range(ns):
                key = frozenset(int(en[e, c]) for c in corners(ctrl_grid[sl]))
                table.setdefault(key, []).append((e, sl))
        recs = sorted((sorted(v) for v in table.values()), key=lambda v: v[0])
        F = len(recs)
        fs.axis = np.zeros(F, dtype=np.int64)
        fs.minus = np.full(F, -1, dtype=np.int64)
        fs.plus = np.full(F, -1, dtype=np.int64)
        fs.ctrl = np.zeros((F, nfc, dim))
        fs.slot_face = np.full((E, ns), -1, dtype=np.int64)
        fs.slot_side = np.zeros((E, ns), dtype=np.int64)
        fs.slot_trace = np.zeros((E, ns, (p + 1) ** (dim - 1)), dtype=np.int64)

        def mirror(g):
            return g[::-1] if dim == 2 else g.T

        for f, rec in enumerate(recs):
            if len(rec) > 2 or (len(rec) == 2 and rec[0][0] == rec[1][0]):
                raise ValueError(f"non-conforming face {rec}")
            (em, sm) = rec[0]
            cg, dgg = ctrl_grid[sm], dg_grid[sm]
            if sm % 2 == 0 and not simplex:
                cg, dgg = mirror(cg), mirror(dgg)
            ids = en[em][cg]                          # face-ordered control point ids
            fs.axis[f] = 0 if simplex else sm // 2
            fs.minus[f] = em
            fs.ctrl[f] = nodes[ids.reshape(-1)]
            fs.slot_face[em, sm] = f
            fs.slot_side[em, sm] = 0
            fs.slot_trace[em, sm] = dgg.reshape(-1)
            if len(rec) == 1:
                continue
            (ep, sp) = rec[1]
            fs.plus[f] = ep
            fs.slot_face[ep, sp] = f
            fs.slot_side[ep, sp] = 1
            # where each face control point sits in the plus slot's grid
            pos = {int(en[ep][c]): loc for loc, c in np.ndenumerate(ctrl_grid[sp])}
            try:
                locs = {loc: pos[int(ids[loc])] for loc in np.ndindex(ids.shape)}
            except KeyError as exc:
                raise ValueError(f"non-conforming face between elements {em} and {ep}") from exc
            # the symmetry as an affine map of normalised face coordinates
            o = np.array(locs[(0,) * (dim - 1)]) / r
            cols = []
            for k in range(dim - 1):
                unit = [0] * (dim - 1)
                unit[k] = r
                cols.append(np.array(locs[tuple(unit)]) / r - o)
            for loc in np.ndindex(ids.shape):
                want = o + sum(cols[k] * (loc[k] / r) for k in range(dim - 1))
                if not np.array_equal(np.rint(want * r).astype(int), np.array(locs[loc])):
                    raise ValueError(f"face {f}: control points do not match a face symmetry")
            tr = np.zeros(dgg.shape, dtype=np.int64)
            for loc in np.ndindex(dgg.shape):
                u = o + sum(cols[k] * (loc[k] / p) for k in range(dim - 1))
                tr[loc] = dg_grid[sp][tuple(np.rint(u * p).astype(int))]
            fs.slot_trace[ep, sp] = tr.reshape(-1)
        if np.any(fs.slot_face < 0):
            raise ValueError("an element slot has no face")
        fs._finish()
        return fs

    @classmethod
    def from_tets(cls, nodes, elem_nodes, r: int, p: int):
        """Faces of a conforming mesh of P_r tetrahedra.  A face is the set of
        its three corner control points; its minus element is the one with
        the smaller index (the only one on the boundary) and the face takes
        that slot's vertex order and triangle coordinates, so N = x_s x x_t
        is the minus element's outward normal.  The plus element's slot
        lists the same three corners in another order: a face node with
        barycentric coordinates c over the minus order has them permuted
        over the plus order, which gives the plus element's node on the same
        point."""
        fs = cls.__new__(cls)
        nodes = np.asarray(nodes, dtype=np.float64)
        en = np.asarray(elem_nodes, dtype=np.int64)
        E, ns = len(en), 4
        fs.dim, fs.r, fs.p, fs.nx = 3, r, p, (E, 1, 1)
        fs.tri_faces = True
        ctrl = [simplex_ref.tet_slot_nodes(r, sl) for sl in range(ns)]
        dgl = [simplex_ref.tet_slot_nodes(p, sl) for sl in range(ns)]
        ccorner = [0, r, len(simplex_ref.lattice(r)) - 1]        # face lattice (0,0), (r,0), (0,r)

        def face_index(k):
            return {(int(a), int(b)): q for q, (a, b) in enumerate(simplex_ref.lattice(k))}

        table = {}
        for e in range(E):
            for sl in range(ns):
                key = frozenset(int(en[e, ctrl[sl][c]]) for c in ccorner)
                table.setdefault(key, []).append((e, sl))
        recs = sorted((sorted(v) for v in table.values()), key=lambda v: v[0])
        F = len(recs)
        nfc = len(simplex_ref.lattice(r))
        fs.axis = np.zeros(F, dtype=np.int64)
        fs.minus = np.full(F, -1, dtype=np.int64)
        fs.plus = np.full(F, -1, dtype=np.int64)
        fs.ctrl = np.zeros((F, nfc, 3))
        fs.slot_face = np.full((E, ns), -1, dtype=np.int64)
        fs.slot_side = np.zeros((E, ns), dtype=np.int64)
        fs.slot_trace = np.zeros((E, ns, len(simplex_ref.lattice(p))), dtype=np.int64)
        fi = {k: face_index(k) for k in (r, p)}
        for f, rec in enumerate(recs):
            if len(rec) > 2 or (len(rec) == 2 and rec[0][0] == rec[1][0]):
                raise ValueError(f"non-conforming face {rec}")
            em, sm = rec[0]
            ids = en[em][ctrl[sm]]
            fs.minus[f] = em
            fs.ctrl[f] = nodes[ids]
            fs.slot_face[em, sm] = f
            fs.slot_side[em, sm] = 0
            fs.slot_trace[em, sm] = dgl[sm]
            if len(rec) == 1:
                continue
            ep, sp = rec[1]
            fs.plus[f] = ep
            fs.slot_face[ep, sp] = f
            fs.slot_side[ep, sp] = 1
            mc = [int(ids[c]) for c in ccorner]
            pc = [int(en[ep][ctrl[sp][c]]) for c in ccorner]
            perm = [pc.index(v) for v in mc]        # minus vertex i is plus vertex perm[i]

            def plus_local(k, q):
                a, b = simplex_ref.lattice(k)[q]
                c = [k - a - b, a, b]
                cp = [0, 0, 0]
                for i in range(3):
                    cp[perm[i]] = c[i]
                return fi[k][(cp[1], cp[2])]
            for q in range(nfc):
                if int(en[ep][ctrl[sp][plus_local(r, q)]]) != int(ids[q]):
                    raise ValueError(f"face {f}: control points of elements {em} and {ep} do not match")
            fs.slot_trace[ep, sp] = [dgl[sp][plus_local(p, q)] for q in range(len(dgl[sp]))]
        if np.any(fs.slot_face < 0):
            raise ValueError("an element slot has no face")
        fs._finish()
        return fs

    # ------------------------------------------------------------------
    def face_of_slot(self, e_idx: np.ndarray, slot: int):
        """Face id and side (0 = element is minus, 1 = plus) of element slot.

        Slot 2a is the element's xi_a = 0 face (element is the plus side),
        slot 2a+1 its xi_a = 1 face (element is the minus side)."""
        a, hi = slot // 2, slot % 2
        ext = [self.nx[b] + (1 if b == a else 0) for b in range(self.dim)]
        fid = np.zeros(len(e_idx[0]), dtype=np.int64)
        s = 1
        for b in range(self.dim):
            v = e_idx[b] + (hi if b == a else 0)
            fid = fid + v * s
            s *= ext[b]
        side = 0 if hi else 1
        return self.axis_offset[a] + fid, side

    def trace_nodes(self, slot: int) -> np.ndarray:
        """Element DG node numbers on a slot, in the face's (s, t) order."""
        p, dim = self.p, self.dim
        a, hi = slot // 2, slot % 2
        others = [b for b in range(dim) if b != a]
        out = []
        for loc in range(self.nf):
            rem = loc
            idx = [0] * dim
            for b in others:
                idx[b] = rem % (p + 1)
                rem //= (p + 1)
            idx[a] = p if hi else 0
            m = 0
            s = 1
            for b in range(dim):
                m += idx[b] * s
                s *= p + 1
            out.append(m)
        return np.array(out)

    # ------------------------------------------------------------------
    def _normals(self, pts: np.ndarray, per_face: bool) -> np.ndarray:
        """Scaled normal N at face parameter points.

        pts: (Q, dim-1) shared points, or (F, Q) per-face points in 2D."""
        dim = self.dim
        if dim == 2:
            s = pts if per_face else np.broadcast_to(pts[:, 0], (self.n_faces, pts.shape[0]))
            _, D = basis.lagrange(self._geo_nodes, s.reshape(-1))
            D = D.reshape(s.shape + (self.r + 1,))
            t = np.einsum("fqb,fba->fqa", D, self.ctrl)
            sgn = np.where(self.axis == 0, 1.0, -1.0)[:, None]
            return np.stack([sgn * t[..., 1], -sgn * t[..., 0]], axis=-1)
        V1s, D1s = basis.lagrange(self._geo_nodes, pts[:, 0])
        V1t, D1t = basis.lagrange(self._geo_nodes, pts[:, 1])
        # control point loc = bs + (r+1)*bt
        Ds = np.einsum("qi,qj->qji", D1s, V1t).reshape(len(pts), -1)
        Dt = np.einsum("qi,qj->qji", V1s, D1t).reshape(len(pts), -1)
        t1 = np.einsum("qm,fma->fqa", Ds, self.ctrl)
        t2 = np.einsum("qm,fma->fqa", Dt, self.ctrl)
        n12 = np.cross(t1, t2)
        return np.where((self.axis == 1)[:, None, None], -n12, n12)

    def _tri_normals(self, pts: np.ndarray) -> np.ndarray:
        """N = x_s x x_t of every triangular face at reference points (Q, 2): (F, Q, 3)."""
        _, G = simplex_ref.lagrange(simplex_ref.geometry_nodes(self.r), self.r, pts)   # (Q, nfc, 2)
        t1 = np.einsum("qm,fma->fqa", G[:, :, 0], self.ctrl)
        t2 = np.einsum("qm,fma->fqa", G[:, :, 1], self.ctrl)
        return np.cross(t1, t2)

    def _setup_tri_rule(self):
        """Fixed composite rule of triangular faces: K x K congruent
        sub-triangles (K = 4), the collapsed Gauss rule of p + r points per
        direction on each (exact where Omega . N keeps its sign)."""
        self.rule3_pts, self.rule3_w = simplex_ref.triangle_composite_rule(KINK_SUBDIV_3D, self.p + self.r)
        self.rule3_phi, _ = simplex_ref.lagrange(simplex_ref.dg_nodes(self.p), self.p, self.rule3_pts)
        self.rule3_N = self._tri_normals(self.rule3_pts)

    def _setup_3d_rule(self):
        K = KINK_SUBDIV_3D
        x1, w1 = basis.gauss_legendre(self.p + self.r)
        xs = np.concatenate([(k + x1) / K for k in range(K)])
        ws = np.concatenate([w1 / K for _ in range(K)])
        S, T = np.meshgrid(xs, xs, indexing="ij")      # S varies slowest
        self.rule3_pts = np.stack([T.reshape(-1), S.reshape(-1)], axis=1)  # s fastest
        self.rule3_w = np.kron(ws, ws)
        V1s, _ = basis.lagrange(self._dg_nodes, self.rule3_pts[:, 0])
        V1t, _ = basis.lagrange(self._dg_nodes, self.rule3_pts[:, 1])
        self.rule3_phi = np.einsum("qi,qj->qji", V1s, V1t).reshape(len(self.rule3_pts), -1)
        self.rule3_N = self._normals(self.rule3_pts, per_face=False)  # (F, Q, 3)

    # ------------------------------------------------------------------
    def _pieces_2d(self, om2: np.ndarray):
        """Breakpoints of [0,1] at the sign changes of g(s) = Omega . N(s)."""
        r = self.r
        F = self.n_faces
        if r == 1:
            return np.tile(np.array([0.0, 1.0]), (F, 1))
        # monomial coefficients of g from its values at r distinct points
        sfit = (np.arange(r) + 0.5) / r
        N = self._normals(sfit[:, None], per_face=False)                    # (F, r, 2)
        gv = N @ om2                                                       # (F, r)
        Vm = np.vander(sfit, r, increasing=True)                            # (r, r)
        coef = np.linalg.solve(Vm, gv.T).T                                  # (F, r)
        roots = np.full((F, r - 1), 2.0)
        if r == 2:
            a0, a1 = coef[:, 0], coef[:, 1]
            with np.errstate(divide="ignore", invalid="ignore"):
                rt = np.where(a1 != 0.0, -a0 / a1, 2.0)
            roots[:, 0] = rt
        elif r == 3:
            c, b, a = coef[:, 0], coef[:, 1], coef[:, 2]
            disc = b * b - 4.0 * a * c
            ok = disc > 0.0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            qq = -0.5 * (b + np.where(b >= 0.0, sq, -sq))
            with np.errstate(divide="ignore", invalid="ignore"):
                r1 = np.where(ok & (a != 0.0), qq / a, 2.0)
                r2 = np.where(ok & (qq != 0.0), c / qq, 2.0)
                lin = np.where(b != 0.0, -c / b, 2.0)
            r1 = np.where(a == 0.0, lin, r1)
            r2 = np.where(a == 0.0, 2.0, r2)
            roots[:, 0], roots[:, 1] = r1, r2
        else:
            for f in range(F):
                rr = np.roots(coef[f, ::-1])
                rr = rr[np.abs(rr.imag) == 0.0].real
                roots[f, :len(rr)] = rr
        roots = np.where((roots > 0.0) & (roots < 1.0), roots, 1.0)
        roots.sort(axis=1)
        return np.concatenate([np.zeros((F, 1)), roots, np.ones((F, 1))], axis=1)

    def _normal_one(self, f: int, s: np.ndarray, t: float = 0.0) -> np.ndarray:
        """N of face f at the points (s_k) (2D) or (s_k, t) (3D), (k, dim)."""
        return self._normal_fast(f, np.asarray(s, dtype=np.float64), t, _Poly1D(self._geo_nodes))

    def _normal_fast(self, f, s, t, geo):
        X = self.ctrl[f]
        if self.dim == 2:
            tg = geo.der(s) @ X
            sgn = 1.0 if self.axis[f] == 0 else -1.0
            return np.stack([sgn * tg[:, 1], -sgn * tg[:, 0]], axis=1)
        n1 = self.r + 1
        Xg = X.reshape(n1, n1, 3)                     # [bt][bs][c]
        Vt, Dt = geo.val(np.array([t]))[0], geo.der(np.array([t]))[0]
        a = np.einsum("qi,ji->jqc" if False else "qi,jic->qjc", geo.der(s), Xg)   # d/ds at each bt row
        b = np.einsum("qi,jic->qjc", geo.val(s), Xg)
        t1 = np.einsum("j,qjc->qc", Vt, a)             # x_s
        t2 = np.einsum("j,qjc->qc", Dt, b)             # x_t
        n12 = np.stack([t1[:, 1] * t2[:, 2] - t1[:, 2] * t2[:, 1],
                        t1[:, 2] * t2[:, 0] - t1[:, 0] * t2[:, 2],
                        t1[:, 0] * t2[:, 1] - t1[:, 1] * t2[:, 0]], axis=1)
        return -n12 if self.axis[f] == 1 else n12

    def _romberg_face(self, f: int, om: np.ndarray, tol: float):
        """(P_plus, P_minus, m_plus, m_minus) of face f by adaptive Romberg."""
        nf = self.nf
        geo, dg = _Poly1D(self._geo_nodes), _Poly1D(self._dg_nodes)

        def values(g, phi):
            gp, gm = np.maximum(g, 0.0), np.maximum(-g, 0.0)
            pp = (gp[:, None, None] * phi[:, :, None] * phi[:, None, :]).reshape(len(g), -1)
            pm = (gm[:, None, None] * phi[:, :, None] * phi[:, None, :]).reshape(len(g), -1)
            return np.concatenate([pp, pm, gp[:, None], gm[:, None]], axis=1)

        if self.tri_faces:
            # collapsed coordinates: (s, t) = (u, v (1 - u)), area element 1 - u
            dgn, geon = simplex_ref.dg_nodes(self.p), simplex_ref.geometry_nodes(self.r)
            X = self.ctrl[f]

            def F(v, u):
                pts = np.stack([np.full(len(v), u), v * (1.0 - u)], axis=1)
                phi, _ = simplex_ref.lagrange(dgn, self.p, pts)
                _, G = simplex_ref.lagrange(geon, self.r, pts)
                N = np.cross(G[:, :, 0] @ X, G[:, :, 1] @ X)
                return values(N @ om, phi) * (1.0 - u)
            out = romberg_square(F, tol)
        elif self.dim == 2:
            def F(s):
                return values(self._normal_fast(f, s, 0.0, geo) @ om, dg.val(s))
            out = romberg(F, 0.0, 1.0, tol)
        else:
            def F(s, t):
                Vt = dg.val(np.array([t]))[0]
                phi = (Vt[None, :, None] * dg.val(s)[:, None, :]).reshape(len(s), -1)   # t slow, s fast
                return values(self._normal_fast(f, s, t, geo) @ om, phi)
            out = romberg_square(F, tol)
        k = nf * nf
        return out[:k].reshape(nf, nf), out[k:2 * k].reshape(nf, nf), out[2 * k], out[2 * k + 1]

    def face_points_physical(self, s: np.ndarray, per_face: bool) -> np.ndarray:
        """Physical coordinates of face parameter points, (F, Q, dim)."""
        if self.dim == 2:
            ss = s if per_face else np.broadcast_to(s[:, 0], (self.n_faces, s.shape[0]))
            V, _ = basis.lagrange(self._geo_nodes, ss.reshape(-1))
            V = V.reshape(ss.shape + (self.r + 1,))
            return np.einsum("fqb,fba->fqa", V, self.ctrl)
        V1s, _ = basis.lagrange(self._geo_nodes, s[:, 0])
        V1t, _ = basis.lagrange(self._geo_nodes, s[:, 1])
        V = np.einsum("qi,qj->qji", V1s, V1t).reshape(len(s), -1)
        return np.einsum("qm,fma->fqa", V, self.ctrl)

    def integrals(self, omega: np.ndarray, inflow_fn=None):
        """(P_plus, P_minus, m_plus, m_minus, m_abs[, L_plus, L_minus]).

        P_* (F, nf, nf); m_plus = int max(g,0), m_minus = int max(-g,0),
        m_abs = int |g| (all over the reference face).  Interior sides below
        the tau threshold are zeroed (see module docstring).  With
        ``inflow_fn(x (..., dim)) -> values`` also the boundary loads
        L_plus[a] = int max(g,0) phi_a f ds_ref and L_minus (max(-g,0))."""
        dim = self.dim
        om = np.asarray(omega, dtype=np.float64)[:dim]
        fvals = None
        if dim == 2:
            bp = self._pieces_2d(om)
            xg, wg = basis.gauss_legendre(face_rule_2d(self.r, self.p))
            s0, s1 = bp[:, :-1], bp[:, 1:]                              # (F, k)
            h = s1 - s0
            s = s0[:, :, None] + h[:, :, None] * xg[None, None, :]      # (F, k, g)
            w = h[:, :, None] * wg[None, None, :]
            s = s.reshape(self.n_faces, -1)
            w = w.reshape(self.n_faces, -1)
            g = self._normals(s, per_face=True) @ om                     # (F, Q)
            V, _ = basis.lagrange(self._dg_nodes, s.reshape(-1))
            phi = V.reshape(s.shape + (self.nf,))
            wp = w * np.maximum(g, 0.0)
            wm = w * np.maximum(-g, 0.0)
            Pp = np.einsum("fq,fqa,fqb->fab", wp, phi, phi)
            Pm = np.einsum("fq,fqa,fqb->fab", wm, phi, phi)
            if inflow_fn is not None:
                fvals = inflow_fn(self.face_points_physical(s, per_face=True))
                Lp = np.einsum("fq,fq,fqa->fa", wp, fvals, phi)
                Lm = np.einsum("fq,fq,fqa->fa", wm, fvals, phi)
        else:
            g = self.rule3_N @ om                                          # (F, Q)
            wp = self.rule3_w[None, :] * np.maximum(g, 0.0)
            wm = self.rule3_w[None, :] * np.maximum(-g, 0.0)
            phi2 = np.einsum("qa,qb->qab", self.rule3_phi, self.rule3_phi).reshape(len(self.rule3_w), -1)
            Pp = (wp @ phi2).reshape(self.n_faces, self.nf, self.nf)
            Pm = (wm @ phi2).reshape(self.n_faces, self.nf, self.nf)
            if inflow_fn is not None:
                fvals = inflow_fn(self.face_points_physical(self.rule3_pts, per_face=False))
                Lp = np.einsum("fq,fq,qa->fa", wp, fvals, self.rule3_phi)
                Lm = np.einsum("fq,fq,qa->fa", wm, fvals, self.rule3_phi)
        mp = wp.sum(axis=1)
        mm = wm.sum(axis=1)
        if self.romberg_tol is not None:
            if dim == 2:
                kink = bp[:, 1] < 1.0
            else:
                kink = (g > 0.0).any(axis=1) & (g < 0.0).any(axis=1)
            # faces along the direction are dropped below: no Romberg there
            kink &= ~(self.interior & (mp + mm <= TAU * self.n_area))
            for f in np.nonzero(kink)[0]:
                Pp[f], Pm[f], mp[f], mm[f] = self._romberg_face(f, om, self.romberg_tol * (mp[f] + mm[f]))
        mabs = mp + mm
        # a face along the direction (int |g| at most tau |int N|: Omega . N
        # vanishes up to rounding) couples nothing; otherwise a side whose
        # measure is at most tau int |g| is dropped
        tangential = self.interior & (mabs <= TAU * self.n_area)
        drop_p = self.interior & ((mp <= TAU * mabs) | tangential)
        drop_m = self.interior & ((mm <= TAU * mabs) | tangential)
        Pp[drop_p] = 0.0
        Pm[drop_m] = 0.0
        mp = np.where(drop_p, 0.0, mp)
        mm = np.where(drop_m, 0.0, mm)
        if fvals is not None:
            return Pp, Pm, mp, mm, mabs, Lp, Lm
        return Pp, Pm, mp, mm, mabs
