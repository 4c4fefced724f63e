"""Pins of the oracle's adaptive Romberg integration (section 2, end: Romberg
for the face integrands that are only piecewise smooth where Omega . n
changes sign).

* The integrator itself: closed-form integrals of a kinked |x - a| and of
  smooth functions, to the requested tolerance; polynomials of degree up to
  5 on one interval without halving.
* 2D faces (quads and triangles): Romberg on every sign-changing face agrees
  with the exact split at the roots of Omega . N (itself pinned against
  scipy's adaptive quadrature) to about the requested tolerance.
* 3D faces of a trilinear mesh: Omega . N is bilinear in the face
  coordinates, so for fixed t the integrand is split exactly at the root in
  s and the outer integral over t is smooth between the values of t where
  that root leaves [0, 1]; Gauss rules on those pieces give a reference to
  rounding, which Romberg meets to its tolerance (and the fixed composite
  rule only to its O(h^2) error at the kink).
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle import basis
from oracle.discretization import Discretization
from oracle.romberg import romberg


def test_romberg_closed_forms():
    for a in (0.3, 1.0 / 3.0, 0.5, 0.9):
        f = lambda x: np.stack([np.abs(x - a), np.maximum(x - a, 0.0) ** 2], axis=1)
        got = romberg(f, 0.0, 1.0, 1e-12)
        want = [0.5 * (a * a + (1 - a) ** 2), (1 - a) ** 3 / 3.0]
        assert np.abs(got - want).max() < 1e-11
    got = romberg(lambda x: np.stack([np.exp(x), np.sin(3 * x)], axis=1), 0.0, 1.0, 1e-13)
    assert abs(got[0] - (math.e - 1)) < 1e-13 and abs(got[1] - (1 - math.cos(3)) / 3) < 1e-13
    # degree 5: T_2,2 is exact, so the first test (row 3) accepts without halving
    calls = []

    def poly(x):
        calls.append(len(x))
        return (x ** 5 - 2 * x ** 3 + x)[:, None]
    got = romberg(poly, 0.0, 1.0, 1e-14)
    assert abs(got[0] - (1 / 6 - 1 / 2 + 1 / 2)) < 1e-15 and sum(calls) == 9


@pytest.mark.parametrize("make", [
    lambda: W.small(dim=2, n=6, r=3, p=2, N=4, amp=0.3 / 6, freq=2),
    lambda: W.annulus_quarter(4, 6, 2, 4),
    lambda: W.tri_annulus(nr=2, nt=8, r=3, p=2, sn_order=4, seed=4),
], ids=["cyclic-q3p2", "annulus-q3p2", "triangles-q3p2"])
def test_romberg_matches_root_split_2d(make):
    wp = make()
    d0 = Discretization(wp)
    d1 = Discretization(replace(wp, face_rule="romberg", face_tol=1e-11))
    n_kink = 0
    for d in range(d0.D):
        a = d0.faces.integrals(d0.omega[d])
        b = d1.faces.integrals(d1.omega[d])
        n_kink += int((d0.faces._pieces_2d(d0.omega[d][:2])[:, 1] < 1.0).sum())
        for x, y in zip(a[:4], b[:4]):
            assert np.abs(x - y).max() <= 2e-11 * np.abs(x).max()
    assert n_kink > 0


def _bilinear_reference(fs, f, om, p, n_gauss=48):
    """Exact-to-rounding P_plus, P_minus of a bilinear face: root split in s,
    Gauss pieces in t between the values where the root crosses s = 0, 1."""
    nf = (p + 1) ** 2
    corners = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    gc = np.array([fs._normal_one(f, np.array([s]), t)[0] @ om for s, t in corners])
    # g(s, t) = c00 + c10 s + c01 t + c11 s t from the corner values
    c00, c10, c01 = gc[0], gc[1] - gc[0], gc[2] - gc[0]
    c11 = gc[3] - gc[1] - gc[2] + gc[0]
    brk = [0.0, 1.0]
    for a0, a1 in ((c00, c01), (c00 + c10, c01 + c11)):      # g(0, t), g(1, t) linear in t
        if a1 != 0.0 and 0.0 < -a0 / a1 < 1.0:
            brk.append(-a0 / a1)
    brk = np.sort(brk)
    xg, wg = basis.gauss_legendre(n_gauss)
    xs, ws = basis.gauss_legendre(p + 2)
    Pp, Pm = np.zeros((nf, nf)), np.zeros((nf, nf))
    for t0, t1 in zip(brk[:-1], brk[1:]):
        for tq, tw in zip(t0 + (t1 - t0) * xg, (t1 - t0) * wg):
            b0, b1 = c00 + c01 * tq, c10 + c11 * tq                # g(s, tq) = b0 + b1 s
            sb = [0.0, 1.0] + ([-b0 / b1] if b1 != 0.0 and 0.0 < -b0 / b1 < 1.0 else [])
            sb = np.sort(sb)
            Vt, _ = basis.lagrange(fs._dg_nodes, np.array([tq]))
            for s0, s1 in zip(sb[:-1], sb[1:]):
                s = s0 + (s1 - s0) * xs
                Vs, _ = basis.lagrange(fs._dg_nodes, s)
                phi = np.einsum("qi,j->qji", Vs, Vt[0]).reshape(len(s), -1)
                g = b0 + b1 * s
                w = tw * (s1 - s0) * ws
                Pp += np.einsum("q,qa,qb->ab", w * np.maximum(g, 0.0), phi, phi)
                Pm += np.einsum("q,qa,qb->ab", w * np.maximum(-g, 0.0), phi, phi)
    return Pp, Pm, (c00, c10, c01, c11)


def gc_scale(fs, f, om):
    return max(abs(fs._normal_one(f, np.array([0.0, 1.0]), 0.0) @ om).max(), 1e-300)


def test_romberg_3d_bilinear_faces():
    wp = W.small(dim=3, n=3, r=1, p=1, N=2, amp=0.08, freq=1)
    d0 = Discretization(wp)
    d1 = Discretization(replace(wp, face_rule="romberg", face_tol=1e-9))
    fs = d0.faces
    checked = 0
    for d in (1, 4):
        om = d0.omega[d]
        g = fs.rule3_N @ om
        kink = np.nonzero((g > 0).any(1) & (g < 0).any(1))[0]
        a = fs.integrals(om)
        b = d1.faces.integrals(om)
        for f in kink:
            Pp, Pm, (c00, c10, c01, c11) = _bilinear_reference(fs, f, om, wp.p)
            scale = np.abs(Pp).max() + np.abs(Pm).max()
            # the reference takes g bilinear from its corner values: so it is
            # (N of a trilinear map is even linear in s and t)
            ss, tt = np.array([0.3, 0.7, 0.55]), 0.4
            g_in = fs._normal_one(f, ss, tt) @ om
            assert np.allclose(g_in, c00 + c10 * ss + c01 * tt + c11 * ss * tt, rtol=0,
                               atol=1e-14 * gc_scale(fs, f, om))
            assert np.abs(b[0][f] - Pp).max() <= 1e-8 * scale
            assert np.abs(b[1][f] - Pm).max() <= 1e-8 * scale
            # the fixed composite rule is only first-order accurate here
            assert np.abs(a[0][f] - Pp).max() <= 1e-2 * scale
            checked += 1
    assert checked >= 4
