"""Pins of the oracle's element geometry and matrices (eqs. Jacobian,
localMtMatrix, localGMatrix)."""
import numpy as np
import pytest

import workloads as W
from oracle.discretization import Discretization
from oracle.geometry import ElementGeometry
from tests.oracle_helpers import exact_int01, gll, lagrange_polys


def one_d_matrices(p):
    L = lagrange_polys(gll(p))
    M1 = np.array([[exact_int01(a * b) for b in L] for a in L])
    C1 = np.array([[exact_int01(a.deriv() * b) for b in L] for a in L])
    return M1, C1


@pytest.mark.parametrize("dim,r,p", [(2, 1, 1), (2, 2, 3), (2, 3, 2), (3, 1, 1), (3, 2, 2)])
def test_unwarped_closed_forms(dim, r, p):
    n = 3
    prob = W.small(dim=dim, n=n, r=r, p=p, N=2, amp=0.0)
    g = ElementGeometry(prob.lattice, dim, prob.nx, r, p)
    h = 1.0 / n
    assert np.allclose(g.J, h * np.eye(dim), atol=1e-14)
    M1, C1 = one_d_matrices(p)
    if dim == 2:
        Mref = h ** 2 * np.kron(M1, M1)
        Kref = [h * np.kron(M1, C1), h * np.kron(C1, M1)]
    else:
        Mref = h ** 3 * np.kron(M1, np.kron(M1, M1))
        Kref = [h ** 2 * np.kron(M1, np.kron(M1, C1)),
                h ** 2 * np.kron(M1, np.kron(C1, M1)),
                h ** 2 * np.kron(C1, np.kron(M1, M1))]
    M = g.mass()
    K = g.grad_moments()
    assert np.allclose(M, Mref[None], atol=1e-15)
    for i in range(dim):
        assert np.allclose(K[:, i], Kref[i][None], atol=1e-14)


@pytest.mark.parametrize("dim,r,p,n,amp,freq,unstructured", [
    (2, 3, 3, 8, 0.3 / 8, 2, None), (2, 2, 1, 5, 0.05, 1, None), (3, 2, 2, 3, 0.05, 1, None),
    (2, 3, 3, 8, 0.3 / 8, 2, 5), (3, 2, 2, 3, 0.05, 1, 6), (3, 1, 2, 3, 0.05, 1, 7)])
def test_warped_invariants(dim, r, p, n, amp, freq, unstructured):
    """Volume, column sums of K_i, and integration by parts on every element
    (K_i + K_i^T = the surface integral of u_m u_n n_i, assembled from the
    element's faces through its slot tables).  With `unstructured` the same
    mesh is given as an element list, renumbered and with every element's
    local frame rotated at random, so each face is assembled through the
    orientation found by face matching."""
    prob = W.small(dim=dim, n=n, r=r, p=p, N=2, amp=amp, freq=freq)
    if unstructured is not None:
        prob = W.as_unstructured(prob, seed=unstructured)
    disc = Discretization(prob)
    assert disc.geo.detJ.min() > 0
    # total volume of the unit box (the warp fixes the boundary)
    assert abs(disc.M.sum() - 1.0) < 1e-13
    # sum_m d(u_m)/dx_i = 0, so the column sums of K_i vanish
    assert np.abs(disc.K.sum(axis=2)).max() < 1e-13
    # integration by parts: K_i + K_i^T = surface integral of u_m u_n n_i
    for i in range(dim):
        om = np.zeros(3)
        om[i] = 1.0
        Pp, Pm, *_ = disc.faces.integrals(om)
        S = np.zeros((disc.E, disc.n, disc.n))
        rows = np.arange(disc.E)[:, None, None]
        for s in range(2 * dim):
            fid = disc.slot_face[:, s]
            sign = np.where(disc.slot_side[:, s] == 0, 1.0, -1.0)[:, None, None]
            tn = disc.slot_trace[:, s]
            S[rows, tn[:, :, None], tn[:, None, :]] += sign * (Pp[fid] - Pm[fid])
        Ki = disc.K[:, i]
        assert np.abs(Ki + Ki.transpose(0, 2, 1) - S).max() < 1e-12 * max(1, np.abs(S).max())


@pytest.mark.parametrize("dim,r,p,n,amp,freq", [(2, 3, 3, (5, 4), 0.3 / 8, 2), (2, 2, 2, (3, 4), 0.05, 1),
                                                 (3, 2, 2, (2, 3, 3), 0.05, 1), (3, 1, 1, (3, 2, 2), 0.02, 1)])
def test_warped_mass_against_independent_jacobian(dim, r, p, n, amp, freq):
    """M_e = int phi_i phi_j |J| on curved elements, recomputed from the
    lattice with independent polynomials and a tensor Gauss rule that is
    exact for the polynomial integrand (the Jacobian determinant of a Q_r map
    has degree dim*r - 1 per axis)."""
    prob = W.small(dim=dim, n=n, r=r, p=p, N=2, amp=amp, freq=freq)
    disc = Discretization(prob)
    nx = prob.nx
    sizes = [r * nx[a] + 1 for a in range(dim)]
    lat = prob.lattice.reshape(tuple(reversed(sizes)) + (dim,))        # [z][y][x] or [y][x]
    G = lagrange_polys(np.linspace(0, 1, r + 1))
    Bp = lagrange_polys(gll(p))
    xq, wq = np.polynomial.legendre.leggauss(p + (dim * r + 1) // 2 + 1)
    xq, wq = (xq + 1) / 2, wq / 2
    Gv = np.array([g(xq) for g in G])                  # (r+1, Q)
    dGv = np.array([g.deriv()(xq) for g in G])
    Bv = np.array([b(xq) for b in Bp])                 # (p+1, Q)
    k = p + 1
    for e in range(disc.E):
        ia = [(e // int(np.prod(nx[:a]))) % nx[a] for a in range(dim)]
        if dim == 2:
            X = lat[ia[1] * r:ia[1] * r + r + 1, ia[0] * r:ia[0] * r + r + 1]          # [b_y][b_x][c]
            jx = np.einsum("bac,aq,br->rqc", X, dGv, Gv)     # d x / d xi  at [eta_r][xi_q]
            jy = np.einsum("bac,aq,br->rqc", X, Gv, dGv)     # d x / d eta
            det = jx[..., 0] * jy[..., 1] - jx[..., 1] * jy[..., 0]
            phi = np.einsum("iq,jr->jirq", Bv, Bv).reshape(k * k, len(xq), len(xq))  # m = i + k j
            w = np.outer(wq, wq)
            Me = np.einsum("mrq,nrq,rq->mn", phi, phi, det * w)
        else:
            X = lat[ia[2] * r:ia[2] * r + r + 1, ia[1] * r:ia[1] * r + r + 1, ia[0] * r:ia[0] * r + r + 1]
            cols = [np.einsum("cbad,aq,br,cs->srqd", X, dGv, Gv, Gv),
                    np.einsum("cbad,aq,br,cs->srqd", X, Gv, dGv, Gv),
                    np.einsum("cbad,aq,br,cs->srqd", X, Gv, Gv, dGv)]
            det = np.linalg.det(np.stack(cols, axis=-1))
            phi = np.einsum("iq,jr,ls->ljisrq", Bv, Bv, Bv).reshape(k ** 3, len(xq), len(xq), len(xq))
            w = np.einsum("s,r,q->srq", wq, wq, wq)
            Me = np.einsum("msrq,nsrq,srq->mn", phi, phi, det * w)
        assert det.min() > 0
        assert np.abs(disc.M[e] - Me).max() <= 1e-13 * np.abs(Me).max(), e
