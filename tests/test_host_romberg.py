"""The library's Romberg face rule (SNSW_FACE_ROMBERG, section 2's adaptive
Romberg for the integrands that change sign) against the oracle, on the CPU:
face integrals through the introspection call, and the graphs it leads to.

* 2D faces (quads, triangles): the library's exact root split equals the
  oracle's to rounding; its Romberg values meet the exact ones, and the
  oracle's Romberg values, to the tolerance.
* 3D faces of a trilinear mesh: the library's Romberg values meet the
  semi-analytic reference of test_oracle_romberg (root split in s, Gauss
  pieces in t) to the tolerance.
* Graphs built with Romberg face matrices equal the oracle's bit for bit.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from oracle.discretization import Discretization
from tests.lib_helpers import graph_parity
from tests.test_oracle_romberg import _bilinear_reference


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_11080_amd import Context
    return Context(device=-1)


@pytest.mark.parametrize("make", [
    lambda: W.small(dim=2, n=6, r=3, p=2, N=4, amp=0.3 / 6, freq=2),
    lambda: W.tri_annulus(nr=2, nt=8, r=3, p=2, sn_order=4, seed=4),
], ids=["quads-q3p2", "triangles-q3p2"])
def test_face_integrals_2d(ctx, make):
    from paper_1810_11080_amd import Problem
    wp = make()
    P0 = Problem.from_workload(ctx, wp)
    P1 = Problem.from_workload(ctx, replace(wp, face_rule="romberg", face_tol=1e-11))
    d0 = Discretization(wp)
    d1 = Discretization(replace(wp, face_rule="romberg", face_tol=1e-11))
    nf = d0.faces.nf
    kinks = 0
    for d in range(d0.D):
        a = d0.faces.integrals(d0.omega[d])
        b = d1.faces.integrals(d1.omega[d])
        bp = d0.faces._pieces_2d(d0.omega[d][:2])
        for f in np.nonzero(bp[:, 1] < 1.0)[0]:
            if d0.faces.interior[f] and a[4][f] <= 1e-12 * d0.faces.n_area[f]:
                continue   # along the direction: dropped
            c0, mp0, mm0, Pp0, Pm0 = P0.face_integrals(d, int(f), nf)
            c1, mp1, mm1, Pp1, Pm1 = P1.face_integrals(d, int(f), nf)
            assert c0 == c1 == 2
            scale = mp0 + mm0
            # exact split: library = oracle to rounding (before any drop)
            assert abs(mp0 - a[2][f]) <= 1e-13 * scale or a[2][f] == 0.0
            assert np.abs(Pp0 - a[0][f]).max() <= 1e-13 * scale or not a[0][f].any()
            # Romberg: to the tolerance, against the exact values and the oracle's Romberg
            assert np.abs(Pp1 - Pp0).max() <= 3e-11 * scale and np.abs(Pm1 - Pm0).max() <= 3e-11 * scale
            assert abs(mp1 - mp0) <= 3e-11 * scale and abs(mm1 - mm0) <= 3e-11 * scale
            if b[2][f] > 0:
                assert np.abs(Pp1 - b[0][f]).max() <= 3e-11 * scale
            kinks += 1
    assert kinks > 0


def test_face_integrals_3d_bilinear(ctx):
    from paper_1810_11080_amd import Problem
    wp = W.small(dim=3, n=3, r=1, p=1, N=2, amp=0.08, freq=1)
    P = Problem.from_workload(ctx, replace(wp, face_rule="romberg", face_tol=1e-10))
    Pe = Problem.from_workload(ctx, wp)
    d0 = Discretization(wp)
    fs = d0.faces
    checked = 0
    for d in range(d0.D):
        om = d0.omega[d]
        g = fs.rule3_N @ om
        for f in np.nonzero((g > 0).any(1) & (g < 0).any(1))[0]:
            Pp, Pm, _ = _bilinear_reference(fs, f, om, wp.p)
            scale = np.abs(Pp).max() + np.abs(Pm).max()
            c, mp, mm, Lp, Lm = P.face_integrals(d, int(f), fs.nf)
            assert c == 2
            assert np.abs(Lp - Pp).max() <= 1e-9 * scale and np.abs(Lm - Pm).max() <= 1e-9 * scale
            # the fixed composite rule: first order at the kink
            c, _, _, Fp, _ = Pe.face_integrals(d, int(f), fs.nf)
            assert np.abs(Fp - Pp).max() <= 1e-2 * scale
            checked += 1
    assert checked >= 8


@pytest.mark.parametrize("make", [
    lambda: W.small(dim=2, n=8, r=3, p=2, N=4, amp=0.3 / 8, freq=2),
    lambda: W.tri_annulus(nr=2, nt=12, r=3, p=2, sn_order=4, seed=6),
], ids=["quads", "triangles"])
def test_romberg_graphs_bit_exact(ctx, make):
    from paper_1810_11080_amd import Problem
    wp = replace(make(), face_rule="romberg", face_tol=1e-10)
    P = Problem.from_workload(ctx, wp)
    bad, _ = graph_parity(P, wp)
    assert bad == []


def test_face_rule_validation(ctx):
    from paper_1810_11080_amd import Problem, SnswError
    wp = W.c1()
    with pytest.raises(SnswError) as ei:
        Problem(ctx, dim=2, nx=wp.nx, geom_order=wp.r, dg_order=wp.p, lattice=wp.lattice, sn_order=2,
                sigma_t=wp.sigma_t, sigma_s=wp.sigma_s, q=wp.q, face_rule=3)
    assert ei.value.code == -1
    with pytest.raises(SnswError) as ei:
        Problem(ctx, dim=2, nx=wp.nx, geom_order=wp.r, dg_order=wp.p, lattice=wp.lattice, sn_order=2,
                sigma_t=wp.sigma_t, sigma_s=wp.sigma_s, q=wp.q, face_rule=1, face_tol=float("nan"))
    assert ei.value.code == -3
    P = Problem.from_workload(ctx, wp)
    with pytest.raises(SnswError):
        P.face_integrals(0, 10 ** 6, 4)


def test_face_integrals_tet_faces(ctx):
    """Triangular faces of curved tetrahedra: the library's composite rule
    equals the oracle's to rounding on every face of two directions, and its
    Romberg values meet the oracle's Romberg values on sign-changing faces
    (one per direction, to keep the oracle's iterated Romberg short) to the
    tolerance."""
    from paper_1810_11080_amd import Problem
    wp = W.tet_shell(nr=1, nt=6, nz=1, r=2, p=1, sn_order=2)
    P0 = Problem.from_workload(ctx, wp)
    P1 = Problem.from_workload(ctx, replace(wp, face_rule="romberg", face_tol=1e-7))
    d0 = Discretization(wp)
    fs = d0.faces
    nf = fs.nf
    checked = 0
    for d in (0, 3):
        om = d0.omega[d]
        a = fs.integrals(om)
        g = fs.rule3_N @ om
        kink = (g > 0).any(1) & (g < 0).any(1)
        for f in range(fs.n_faces):
            c0, mp0, mm0, Pp0, Pm0 = P0.face_integrals(d, f, nf)
            assert c0 == (2 if kink[f] else (0 if mm0 == 0.0 else 1))
            scale = max(mp0 + mm0, 1e-300)
            assert abs(mp0 - a[2][f]) <= 1e-13 * scale or a[2][f] == 0.0 or a[3][f] == 0.0
            if kink[f] and a[2][f] > 0 and a[3][f] > 0:
                assert np.abs(Pp0 - a[0][f]).max() <= 1e-13 * scale
        for f in np.nonzero(kink & ~(fs.interior & (a[4] <= 1e-12 * fs.n_area)))[0][:1]:
            c1, mp1, mm1, Pp1, Pm1 = P1.face_integrals(d, int(f), nf)
            ref = fs._romberg_face(int(f), om, 1e-7 * (a[2][f] + a[3][f]))
            scale = a[2][f] + a[3][f]
            assert np.abs(Pp1 - ref[0]).max() <= 1e-6 * scale and np.abs(Pm1 - ref[1]).max() <= 1e-6 * scale
            checked += 1
    assert checked >= 2
