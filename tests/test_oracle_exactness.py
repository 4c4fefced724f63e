"""Exactness pins of the oracle's discretisation and sweep.

* constant solutions: sigma_s = 0, q = sigma_t C, psi_inc = C gives psi = C
  on any curved mesh (pins the signs of the face terms, the printed
  eqs. offDiagonalFaceMatrixBlocks/qVectorDef being read with the sign of the
  integration by parts);
* linear solutions a + b.x lie in the DG space when p >= r, so the discrete
  solution reproduces them (pins the streaming matrix, eq. localGMatrix, and
  its orientation);
* method of manufactured solutions with the paper's manufactured flux (eq.
  psiAnnularMMS) on warped squares: the scalar-flux L2 error decays at about
  order p+1.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, source_iteration


@pytest.mark.parametrize("dim,n,r,p,N,amp,freq", [
    (2, 8, 3, 3, 8, 0.3 / 8, 2),      # cyclic graph (C2-like warp)
    (2, 6, 2, 2, 4, 0.05, 1),
    (3, 3, 2, 2, 4, 0.05, 1),
    (3, 3, 1, 1, 2, 0.03, 1),
])
def test_constant_solution(dim, n, r, p, N, amp, freq):
    C = 1.7
    E = n ** dim
    st = np.linspace(0.3, 3.0, E)
    prob = W.small(dim=dim, n=n, r=r, p=p, N=N, amp=amp, freq=freq, sigma_t=st, c=0.0,
                   q=st * C, bc_kind=W.ISO_CONST, psi_inc=C)
    disc = Discretization(prob)
    gs = build_graphs(disc)
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-15, max_iters=60)
    assert np.abs(psi - C).max() < 1e-11


@pytest.mark.parametrize("dim,n,r,p,N,c", [(2, 5, 2, 2, 4, 0.0), (2, 4, 3, 3, 4, 0.6),
                                           (2, 6, 1, 1, 4, 0.3), (3, 3, 2, 2, 2, 0.5)])
def test_linear_solution(dim, n, r, p, N, c):
    a0 = 0.7
    bvec = np.array([0.4, -0.9, 0.3])[:dim]
    st = 1.3
    ss = c * st

    def psi_fn(x, om):
        return a0 + x @ bvec

    def src(x, om):
        # isotropic linear psi: phi = 4 pi psi, so q = Omega.b + (st - ss) psi
        return np.dot(om[:dim], bvec) + (st - ss) * psi_fn(x, om)

    amp = 0.3 / n if dim == 2 else 0.04
    prob = W.small(dim=dim, n=n, r=r, p=p, N=N, amp=amp, freq=1, sigma_t=st, c=c, q=0.0)
    disc = Discretization(prob, source_fn=src, inflow_fn=psi_fn)
    xn = disc.geo.dg_node_positions()
    exact = a0 + xn @ bvec
    gs = build_graphs(disc)
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-15, max_iters=200)
    assert np.abs(psi - exact[None]).max() < 1e-10
    if disc.D * disc.E * disc.n <= 4000:
        phid, psid = dense.solve(disc)
        assert np.abs(psid - exact[None]).max() < 1e-10


def mms_error(n, p):
    st, c = 1.0, 0.5
    ss = c * st

    def f(x):
        return 0.5 * (1 + x[..., 0] ** 2 + x[..., 1] ** 2) + np.cos(3 * x[..., 0] + 1.5 * x[..., 1])

    def gradf(x):
        sn = np.sin(3 * x[..., 0] + 1.5 * x[..., 1])
        return np.stack([x[..., 0] - 3 * sn, x[..., 1] - 1.5 * sn], axis=-1)

    prob = W.small(dim=2, n=n, r=2, p=p, N=4, amp=0.05, freq=1, sigma_t=st, c=c, q=0.0)
    from oracle.quadrature import level_symmetric
    om, w = level_symmetric(4, 2)
    Aang = np.dot(w, om[:, 0] ** 2 + om[:, 1])

    def psi_fn(x, o):
        return f(x) * (o[0] ** 2 + o[1])

    def src(x, o):
        a = o[0] ** 2 + o[1]
        return a * (gradf(x) @ o[:2]) + st * a * f(x) - ss / (4 * np.pi) * Aang * f(x)

    disc = Discretization(prob, source_fn=src, inflow_fn=psi_fn)
    gs = build_graphs(disc)
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-13, max_iters=300)
    from oracle.geometry import ElementGeometry
    fine = ElementGeometry(prob.lattice, 2, prob.nx, 2, p, extra_points=4)
    phih = np.einsum("en,qn->eq", phi, fine.U)
    err2 = np.einsum("q,eq,eq->", fine.wq, fine.detJ, (phih - Aang * f(fine.x)) ** 2)
    return np.sqrt(err2)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mms_convergence(p):
    ns = [4, 8, 16]
    errs = [mms_error(n, p) for n in ns]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert rates[-1] > p + 0.4, (errs, rates)


def mms_error_nodal(n, p):
    """The same manufactured problem with the source and the incident flux
    given by their values at the DG nodes (per direction), as the library
    takes them."""
    import dataclasses
    from oracle.geometry import ElementGeometry
    from oracle.quadrature import level_symmetric
    st, ss = 1.0, 0.5
    prob = W.small(dim=2, n=n, r=2, p=p, N=4, amp=0.05, freq=1, sigma_t=st, c=ss / st, q=0.0)
    om, w = level_symmetric(4, 2)
    g = ElementGeometry(prob.lattice, 2, prob.nx, 2, p)
    q, psi_exact, _ = W.mms_annular(g.dg_node_positions(), om, w, st, ss)
    prob = dataclasses.replace(prob, q_dir=q, psi_inc_tab=psi_exact, bc_kind=W.TABULATED)
    disc = Discretization(prob)
    gs = build_graphs(disc)
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-13, max_iters=300)
    fine = ElementGeometry(prob.lattice, 2, prob.nx, 2, p, extra_points=4)
    _, _, phi_exact = W.mms_annular(fine.x, om, w, st, ss)
    phih = np.einsum("en,qn->eq", phi, fine.U)
    return np.sqrt(np.einsum("q,eq,eq->", fine.wq, fine.detJ, (phih - phi_exact) ** 2))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mms_convergence_nodal_data(p):
    """Nodal (interpolated) source and tabulated inflow keep order p+1."""
    ns = [4, 8, 16]
    errs = [mms_error_nodal(n, p) for n in ns]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert rates[-1] > p + 0.4, (errs, rates)


@pytest.mark.parametrize("dim,n,r,p,N,amp,freq", [(2, 5, 3, 2, 8, 0.3 / 5, 2), (3, 3, 2, 2, 4, 0.07, 1)])
def test_constant_solution_tabulated(dim, n, r, p, N, amp, freq):
    """psi = C per direction (C_d differs between directions), sigma_s = 0:
    source sigma_t C_d at every node and tabulated inflow C_d reproduce
    psi_d = C_d exactly on a curved mesh (the boundary term of eq. qVectorDef
    taken from tabulated nodal values)."""
    import dataclasses
    prob = W.small(dim=dim, n=n, r=r, p=p, N=N, amp=amp, freq=freq, sigma_t=1.0, c=0.0, q=0.0)
    E, nd = prob.n_elements, prob.n_dof
    D = prob.n_dirs
    st = np.linspace(0.5, 2.0, E)
    Cd = 1.0 + 0.1 * np.arange(D)
    q = Cd[:, None, None] * st[None, :, None] * np.ones((D, E, nd))
    tab = Cd[:, None, None] * np.ones((D, E, nd))
    prob = dataclasses.replace(prob, sigma_t=st, sigma_s=np.zeros(E), q_dir=q, psi_inc_tab=tab,
                               bc_kind=W.TABULATED)
    disc = Discretization(prob)
    gs = build_graphs(disc)
    _, psi, _, _ = source_iteration(disc, gs, tol=1e-15, max_iters=200)
    assert np.abs(psi - Cd[:, None, None]).max() < 1e-10
