"""Pins of the oracle's simplicial elements (section 2: P_r triangles for the
mesh map and P_p for the flux).

* The reference element: the nodal basis is the Lagrange basis of its nodes
  (Kronecker delta, partition of unity, reproduction of P_p); the collapsed
  Gauss rule integrates the monomials xi^a eta^b with the closed form
  a! b! / (a + b + 2)!.
* Affine triangles: the P1 and P2 mass matrices equal their textbook closed
  forms (area / 12 (1 + delta) and the 6 / -1 / -4 / 32 / 16 table over 180).
* Curved triangles: the mesh area (exact where the map fixes the boundary),
  column sums of K_i, linear exactness of K, and integration by parts
  K_i + K_i^T = surface integral of u_m u_n n_i assembled from the face
  integrals through the slot tables (volume and face code checked against
  each other).
* Faces: the two sides of every interior face list DG nodes at the same
  physical points in the face order.
* The discrete solution reproduces any linear angular flux exactly (source
  Omega . b + sigma_t (a + b . x) and tabulated inflow at the nodes), on
  curved meshes whose faces have sign changes of Omega . n: this pins the
  streaming, upwind face and source terms together with their signs.
* Renumbering elements and turning their local frames does not change the
  discrete solution.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, simplex
from oracle.basis import gll_points
from oracle.discretization import Discretization
from oracle.sweep import source_iteration


@pytest.mark.parametrize("k", [1, 2, 3])
def test_nodal_basis(k):
    nodes = simplex.dg_nodes(k)
    V, G = simplex.lagrange(nodes, k, nodes)
    assert np.allclose(V, np.eye(len(nodes)), atol=1e-13)
    pts = np.random.default_rng(k).dirichlet(np.ones(3), size=40)[:, :2]
    V, G = simplex.lagrange(nodes, k, pts)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(G.sum(axis=1), 0.0, atol=1e-12)
    # reproduces xi^a eta^b, a + b <= k, and its gradient
    for a in range(k + 1):
        for b in range(k + 1 - a):
            f = nodes[:, 0] ** a * nodes[:, 1] ** b
            x, y = pts[:, 0], pts[:, 1]
            assert np.allclose(V @ f, x ** a * y ** b, atol=1e-12)
            gx = a * x ** max(a - 1, 0) * y ** b if a else 0 * x
            gy = b * x ** a * y ** max(b - 1, 0) if b else 0 * y
            assert np.allclose(G[:, :, 0] @ f, gx, atol=1e-11)
            assert np.allclose(G[:, :, 1] @ f, gy, atol=1e-11)
    # the GLL lattice: edge nodes at the Gauss-Lobatto points of each edge
    for s in range(3):
        sn = simplex.slot_nodes(k, s)
        v = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
        a, b = v[s], v[(s + 1) % 3]
        want = a[None] + gll_points(k)[:, None] * (b - a)[None]
        assert np.allclose(nodes[sn], want, atol=1e-15)


@pytest.mark.parametrize("nq", [1, 2, 3, 5])
def test_collapsed_rule_monomials(nq):
    x, w = simplex.collapsed_rule(nq)
    for a in range(2 * nq - 1):
        for b in range(2 * nq - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(w * x[:, 0] ** a * x[:, 1] ** b) - exact) < 1e-15


def _affine_triangle(seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, 2))
    if (A[1] - A[0])[0] * (A[2] - A[0])[1] - (A[1] - A[0])[1] * (A[2] - A[0])[0] < 0:
        A = A[[0, 2, 1]]
    return A


@pytest.mark.parametrize("p", [1, 2])
def test_affine_mass_closed_form(p):
    A = _affine_triangle(p)
    area = 0.5 * ((A[1] - A[0])[0] * (A[2] - A[0])[1] - (A[1] - A[0])[1] * (A[2] - A[0])[0])
    xe = A[0] + simplex.geometry_nodes(1) @ np.stack([A[1] - A[0], A[2] - A[0]])   # r = 1 control points
    g = simplex.SimplexGeometry(xe[None], 1, p)
    M = g.mass()[0]
    if p == 1:
        ref = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
    else:
        # nodes of order 2: vertices (0,0),(2,0),(0,2) and edge midpoints
        L = simplex.lattice(2)
        vert = {(0, 0): 0, (2, 0): 1, (0, 2): 2}
        kind = []
        for i, j in L:
            if (int(i), int(j)) in vert:
                kind.append(("v", vert[(int(i), int(j))]))
            else:
                # the edge between the two vertices whose barycentric is 1/2
                lam = {0: 2 - i - j, 1: i, 2: j}
                kind.append(("e", frozenset(v for v in range(3) if lam[v] == 1)))
        ref = np.zeros((6, 6))
        for m, km in enumerate(kind):
            for n, kn in enumerate(kind):
                if km[0] == "v" and kn[0] == "v":
                    ref[m, n] = 6 if m == n else -1
                elif km[0] == "e" and kn[0] == "e":
                    ref[m, n] = 32 if m == n else 16
                else:
                    v, e = (km[1], kn[1]) if km[0] == "v" else (kn[1], km[1])
                    ref[m, n] = -4 if v not in e else 0
        ref *= area / 180.0
    assert np.abs(M - ref).max() < 1e-14 * max(1.0, abs(area))


@pytest.mark.parametrize("make", [
    lambda: W.tri_square(n=3, r=2, p=2, seed=3),
    lambda: W.tri_square(n=2, r=3, p=3, amp=0.06, seed=4),
    lambda: W.tri_square(n=3, r=1, p=1, seed=None),
    lambda: W.tri_annulus(nr=2, nt=8, r=3, p=2, seed=1),
    lambda: W.tri_annulus(nr=2, nt=6, r=2, p=3, seed=2),
], ids=["square-q2p2", "square-q3p3", "square-q1p1", "annulus-q3p2", "annulus-q2p3"])
def test_curved_invariants(make):
    prob = make()
    disc = Discretization(prob)
    assert disc.geo.detJ.min() > 0
    if prob.name.startswith("tri_square"):
        assert abs(disc.M.sum() - 1.0) < 1e-13            # the warp fixes the unit square's boundary
    else:
        # annulus: the order-r interpolant of the circles (converges to 3 pi,
        # test_annulus_area_converges)
        assert abs(disc.M.sum() - 3.0 * math.pi) < 3e-2
    assert np.abs(disc.K.sum(axis=2)).max() < 1e-13
    # linear exactness (x lies in the DG space when r <= p):
    # sum_m x_i(node m) K_j[m, n] = delta_ij sum_m M[m, n]
    xn = disc.geo.dg_node_positions()
    if prob.r <= prob.p:
        for i in range(2):
            for j in range(2):
                lhs = np.einsum("em,emn->en", xn[:, :, i], disc.K[:, j])
                rhs = disc.M.sum(axis=1) if i == j else 0.0 * lhs
                assert np.abs(lhs - rhs).max() < 1e-12
    # integration by parts through the face integrals and slot tables
    for i in range(2):
        om = np.zeros(3)
        om[i] = 1.0
        Pp, Pm, *_ = disc.faces.integrals(om)
        S = np.zeros((disc.E, disc.n, disc.n))
        rows = np.arange(disc.E)[:, None, None]
        for s in range(disc.ns):
            fid = disc.slot_face[:, s]
            sign = np.where(disc.slot_side[:, s] == 0, 1.0, -1.0)[:, None, None]
            tn = disc.slot_trace[:, s]
            S[rows, tn[:, :, None], tn[:, None, :]] += sign * (Pp[fid] - Pm[fid])
        Ki = disc.K[:, i]
        assert np.abs(Ki + Ki.transpose(0, 2, 1) - S).max() < 1e-12 * max(1, np.abs(S).max())
    # both sides of an interior face put their trace nodes on the same points
    fs = disc.faces
    for f in np.nonzero(fs.interior)[0]:
        em, ep = fs.minus[f], fs.plus[f]
        sm = int(np.nonzero(disc.slot_face[em] == f)[0][0])
        sp = int(np.nonzero(disc.slot_face[ep] == f)[0][0])
        assert np.allclose(xn[em, disc.slot_trace[em, sm]], xn[ep, disc.slot_trace[ep, sp]], atol=1e-13)
    assert fs.n_faces == (3 * disc.E + (~fs.interior).sum()) // 2


@pytest.mark.parametrize("r", [2, 3])
def test_annulus_area_converges(r):
    """The area of the order-r triangulated annulus tends to 3 pi at least as
    fast as the interpolation error of the circles, h^(r+1)."""
    err = [abs(Discretization(W.tri_annulus(nr=2, nt=nt, r=r, p=1, seed=None)).M.sum() - 3.0 * math.pi)
           for nt in (12, 24)]
    assert err[0] / err[1] > 0.8 * 2.0 ** (r + 1)


@pytest.mark.parametrize("make", [
    lambda: W.tri_square(n=2, r=1, p=1, seed=3),
    lambda: W.tri_square(n=2, r=2, p=2, amp=0.06, seed=4),
    lambda: W.tri_annulus(nr=2, nt=6, r=2, p=2, seed=1),
    lambda: W.tri_annulus(nr=1, nt=6, r=3, p=3, seed=2),
    lambda: W.tri_annulus(nr=1, nt=8, r=2, p=3, seed=5),
], ids=["square-q1p1", "square-q2p2", "annulus-q2p2", "annulus-q3p3", "annulus-q2p3"])
def test_linear_solution_reproduced(make):
    """psi_d(x) = a_d + b_d . x solves Omega_d . grad psi + sigma_t psi = q_d
    with q_d = Omega_d . b_d + sigma_t psi_d.  On order-r triangles with
    r <= p it lies in the DG space (x itself is a polynomial of degree r in
    the reference coordinates), so the upwind DG solution (eq.
    matrixFormLinearTransport with the inflow of eq. qVectorDef given at the
    nodes) equals it exactly."""
    prob = make()
    prob.sigma_s[:] = 0.0
    disc0 = Discretization(prob)
    xn = disc0.geo.dg_node_positions()                    # (E, n, 2)
    rng = np.random.default_rng(11)
    D = disc0.D
    a = rng.uniform(0.5, 1.5, D)
    b = rng.uniform(-0.3, 0.3, (D, 2))
    psi_exact = a[:, None, None] + np.einsum("dc,enc->den", b, xn)
    om = disc0.omega[:, :2]
    q_dir = np.einsum("dc,dc->d", om, b)[:, None, None] + prob.sigma_t[None, :, None] * psi_exact
    prob.q_dir = q_dir
    prob.bc_kind = W.TABULATED
    prob.psi_inc_tab = psi_exact
    disc = Discretization(prob)
    _, psi = dense.solve(disc)
    assert np.abs(psi - psi_exact).max() < 1e-11 * np.abs(psi_exact).max()
    # the lagged source iteration reaches the same fixed point
    _, psi_si, _, _ = source_iteration(disc, tol=1e-14, max_iters=200)
    phi_si = np.einsum("d,den->en", disc.w, psi_si)
    phi_ex = np.einsum("d,den->en", disc.w, psi_exact)
    assert np.abs(phi_si - phi_ex).max() < 1e-11 * np.abs(phi_ex).max()


@pytest.mark.parametrize("maker", [lambda s: W.tri_square(n=3, r=2, p=2, seed=s),
                                   lambda s: W.tri_square(n=2, r=3, p=3, seed=s),
                                   lambda s: W.tri_annulus(nr=2, nt=6, r=3, p=1, seed=s)],
                         ids=["square-p2", "square-p3", "annulus-p1"])
def test_numbering_and_frames_do_not_matter(maker):
    """The same triangles renumbered with turned local frames: the exact
    discrete solutions agree after mapping elements and nodes back."""
    p0, p1 = maker(None), maker(9)
    phi0, _ = dense.solve(Discretization(p0))
    phi1, _ = dense.solve(Discretization(p1))
    perm, turns = p1.meta["perm"], p1.meta["turns"]
    maps = [W.tri_rotation_map(p0.p, t) for t in range(3)]
    back = np.stack([phi0[perm[k]][maps[turns[k]]] for k in range(len(perm))])
    assert np.abs(phi1 - back).max() < 1e-12 * np.abs(back).max()


# ----------------------------------------------------------------- tetrahedra
@pytest.mark.parametrize("k", [1, 2, 3])
def test_tet_nodal_basis(k):
    nodes = simplex.tet_dg_nodes(k)
    assert len(nodes) == simplex.tet_n_nodes(k)
    V, G = simplex.tet_lagrange(nodes, k, nodes)
    assert np.allclose(V, np.eye(len(nodes)), atol=1e-12)
    pts = np.random.default_rng(k).dirichlet(np.ones(4), size=40)[:, :3]
    V, G = simplex.tet_lagrange(nodes, k, pts)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-12)
    assert np.allclose(G.sum(axis=1), 0.0, atol=1e-11)
    x, y, z = pts.T
    for a in range(k + 1):
        for b in range(k + 1 - a):
            for c in range(k + 1 - a - b):
                f = nodes[:, 0] ** a * nodes[:, 1] ** b * nodes[:, 2] ** c
                assert np.allclose(V @ f, x ** a * y ** b * z ** c, atol=1e-11)
    # every face carries the triangle's DG node set, placed on that face
    tri = simplex.dg_nodes(k)
    Vt = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    for s in range(4):
        A, B, C = simplex.TET_FACES[s]
        want = Vt[A][None] + tri[:, :1] * (Vt[B] - Vt[A])[None] + tri[:, 1:] * (Vt[C] - Vt[A])[None]
        assert np.allclose(nodes[simplex.tet_slot_nodes(k, s)], want, atol=1e-15)
        # outward: the face normal (B - A) x (C - A) points away from the opposite vertex
        nrm = np.cross(Vt[B] - Vt[A], Vt[C] - Vt[A])
        assert nrm @ (Vt[s] - Vt[A]) < 0


@pytest.mark.parametrize("nq", [1, 2, 3])
def test_tet_collapsed_rule_monomials(nq):
    x, w = simplex.tet_collapsed_rule(nq)
    for a in range(2 * nq - 2):
        for b in range(2 * nq - 2 - a):
            for c in range(2 * nq - 2 - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                assert abs(np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c) - exact) < 1e-15


def test_tet_affine_mass_closed_form():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(4, 3))
    if np.linalg.det(A[1:] - A[0]) < 0:
        A = A[[0, 2, 1, 3]]
    vol = np.linalg.det(A[1:] - A[0]) / 6.0
    xe = A[0] + simplex.tet_geometry_nodes(1) @ (A[1:] - A[0])
    M = simplex.TetGeometry(xe[None], 1, 1).mass()[0]
    assert np.abs(M - vol / 20.0 * (np.ones((4, 4)) + np.eye(4))).max() < 1e-14 * max(1.0, vol)


@pytest.mark.parametrize("make", [
    lambda: W.tet_cube(n=2, r=2, p=2, seed=3),
    lambda: W.tet_cube(n=1, r=3, p=3, amp=0.05, seed=4),
    lambda: W.tet_cube(n=2, r=1, p=1, seed=None),
    lambda: W.tet_shell(nr=1, nt=6, nz=1, r=2, p=1, seed=1),
    lambda: W.tet_shell(nr=1, nt=6, nz=1, r=1, p=2, seed=2),
], ids=["cube-q2p2", "cube-q3p3", "cube-q1p1", "shell-q2p1", "shell-q1p2"])
def test_tet_curved_invariants(make):
    prob = make()
    disc = Discretization(prob)
    assert disc.geo.detJ.min() > 0
    if prob.name.startswith("tet_cube"):
        assert abs(disc.M.sum() - 1.0) < 1e-13            # the warp fixes the cube's boundary
    assert np.abs(disc.K.sum(axis=2)).max() < 1e-13
    xn = disc.geo.dg_node_positions()
    if prob.r <= prob.p:
        for i in range(3):
            for j in range(3):
                lhs = np.einsum("em,emn->en", xn[:, :, i], disc.K[:, j])
                rhs = disc.M.sum(axis=1) if i == j else 0.0 * lhs
                assert np.abs(lhs - rhs).max() < 1e-12
    for i in range(3):
        om = np.zeros(3)
        om[i] = 1.0
        Pp, Pm, *_ = disc.faces.integrals(om)
        S = np.zeros((disc.E, disc.n, disc.n))
        rows = np.arange(disc.E)[:, None, None]
        for s in range(disc.ns):
            fid = disc.slot_face[:, s]
            sign = np.where(disc.slot_side[:, s] == 0, 1.0, -1.0)[:, None, None]
            tn = disc.slot_trace[:, s]
            S[rows, tn[:, :, None], tn[:, None, :]] += sign * (Pp[fid] - Pm[fid])
        Ki = disc.K[:, i]
        assert np.abs(Ki + Ki.transpose(0, 2, 1) - S).max() < 1e-12 * max(1, np.abs(S).max())
    fs = disc.faces
    for f in np.nonzero(fs.interior)[0]:
        em, ep = fs.minus[f], fs.plus[f]
        sm = int(np.nonzero(disc.slot_face[em] == f)[0][0])
        sp = int(np.nonzero(disc.slot_face[ep] == f)[0][0])
        assert np.allclose(xn[em, disc.slot_trace[em, sm]], xn[ep, disc.slot_trace[ep, sp]], atol=1e-13)
    assert fs.n_faces == (4 * disc.E + (~fs.interior).sum()) // 2


@pytest.mark.parametrize("make", [
    lambda: W.tet_cube(n=1, r=1, p=1, seed=3),
    lambda: W.tet_cube(n=1, r=2, p=2, amp=0.05, seed=4),
    lambda: W.tet_shell(nr=1, nt=6, nz=1, r=2, p=2, seed=5),
], ids=["cube-q1p1", "cube-q2p2", "shell-q2p2"])
def test_tet_linear_solution_reproduced(make):
    """As for triangles: a linear angular flux (r <= p) with its manufactured
    source and tabulated inflow is the exact discrete solution on curved
    tetrahedra, faces with sign changes of Omega . N included."""
    prob = make()
    prob.sigma_s[:] = 0.0
    disc0 = Discretization(prob)
    xn = disc0.geo.dg_node_positions()
    rng = np.random.default_rng(13)
    D = disc0.D
    a = rng.uniform(0.5, 1.5, D)
    b = rng.uniform(-0.3, 0.3, (D, 3))
    psi_exact = a[:, None, None] + np.einsum("dc,enc->den", b, xn)
    prob.q_dir = np.einsum("dc,dc->d", disc0.omega, b)[:, None, None] + prob.sigma_t[None, :, None] * psi_exact
    prob.bc_kind = W.TABULATED
    prob.psi_inc_tab = psi_exact
    disc = Discretization(prob)
    _, psi = dense.solve(disc)
    assert np.abs(psi - psi_exact).max() < 1e-11 * np.abs(psi_exact).max()


def test_tet_numbering_and_frames_do_not_matter():
    p0, p1 = W.tet_cube(n=1, r=2, p=2, seed=None), W.tet_cube(n=1, r=2, p=2, seed=9)
    phi0, _ = dense.solve(Discretization(p0))
    phi1, _ = dense.solve(Discretization(p1))
    perm, rot = p1.meta["perm"], p1.meta["rot"]
    evens = W.tet_even_permutations()
    back = np.stack([phi0[perm[k]][W.tet_rotation_map(p0.p, evens[rot[k]])] for k in range(len(perm))])
    assert np.abs(phi1 - back).max() < 1e-12 * np.abs(back).max()
