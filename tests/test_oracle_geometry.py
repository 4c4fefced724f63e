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


@pytest.mark.parametrize("dim,r,p,n,amp,freq", [(2, 3, 3, 8, 0.3 / 8, 2), (2, 2, 1, 5, 0.05, 1),
                                                 (3, 2, 2, 3, 0.05, 1)])
def test_warped_invariants(dim, r, p, n, amp, freq):
    prob = W.small(dim=dim, n=n, r=r, p=p, N=2, amp=amp, freq=freq)
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
        for s in range(2 * dim):
            fid = disc.slot_face[:, s]
            sign = 1.0 if disc.slot_side[s] == 0 else -1.0
            tn = disc.slot_nodes[s]
            S[:, tn[:, None], tn[None, :]] += sign * (Pp[fid] - Pm[fid])
        Ki = disc.K[:, i]
        assert np.abs(Ki + Ki.transpose(0, 2, 1) - S).max() < 1e-12 * max(1, np.abs(S).max())
