"""Pins of the oracle's level-symmetric quadrature (section 2, below eq.
linearSnTransport: positive weights summing to 4 pi; S_2 cosine a = sqrt(3)/3,
Tables 5-7)."""
import math
import os

import numpy as np
import pytest

from oracle import quadrature as Q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "s2_directions.txt")


@pytest.mark.parametrize("N,dim,D", [(2, 2, 4), (4, 2, 12), (8, 2, 40), (2, 3, 8),
                                     (4, 3, 24), (8, 3, 80), (12, 3, 168)])
def test_counts_weights(N, dim, D):
    om, w = Q.level_symmetric(N, dim)
    assert om.shape == (D, 3) and w.shape == (D,)
    assert np.all(w > 0)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    assert np.allclose(np.linalg.norm(om, axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("N", [2, 4, 6, 8, 10, 12])
def test_sphere_moments_3d(N):
    """Closed-form sphere moments: int Omega_x^(2m) = 4 pi/(2m+1) for m < N/2,
    odd moments vanish, second moments are 4 pi/3 delta_ij."""
    om, w = Q.level_symmetric(N, 3)
    for i in range(3):
        assert abs(np.dot(w, om[:, i])) < 1e-13
        assert abs(np.dot(w, om[:, i] ** 3)) < 1e-13
        for m in range(N // 2):
            assert abs(np.dot(w, om[:, i] ** (2 * m)) - 4 * math.pi / (2 * m + 1)) < 1e-12
    sec = np.einsum("d,di,dj->ij", w, om, om)
    assert np.allclose(sec, 4 * math.pi / 3 * np.eye(3), atol=1e-12)


@pytest.mark.parametrize("N", [4, 8, 12])
def test_level_symmetry(N):
    """The set is invariant under axis permutations and reflections."""
    om, w = Q.level_symmetric(N, 3)
    key = {tuple(np.round(o, 12)): ww for o, ww in zip(om, w)}
    for perm in ([1, 0, 2], [2, 1, 0], [0, 2, 1]):
        for o, ww in zip(om, w):
            k = tuple(np.round(o[perm], 12))
            assert k in key and abs(key[k] - ww) < 1e-13


def test_2d_half_sphere():
    om, w = Q.level_symmetric(8, 2)
    assert np.all(om[:, 2] > 0)
    assert abs(np.dot(w, om[:, 0])) < 1e-13 and abs(np.dot(w, om[:, 1])) < 1e-13
    assert abs(np.dot(w, om[:, 0] ** 2) - 4 * math.pi / 3) < 1e-12


def test_s2_matches_paper_table():
    a = math.sqrt(3.0) / 3.0
    signs = np.loadtxt(GOLDEN)
    om, w = Q.level_symmetric(2, 3)
    got = {tuple(np.round(o / a, 12)) for o in om}
    want = {tuple(s) for s in signs}
    assert got == want
    assert np.allclose(w, 4 * math.pi / 8)


def test_direction_order():
    """Octant-major order: o = [x<0] + 2[y<0] + 4[z<0]."""
    om, _ = Q.level_symmetric(8, 3)
    per = 80 // 8
    for d in range(80):
        o = d // per
        assert (om[d, 0] < 0) == bool(o & 1)
        assert (om[d, 1] < 0) == bool(o & 2)
        assert (om[d, 2] < 0) == bool(o & 4)


# mu_1 of the level-symmetric sets as printed in the transport literature
# (Lewis and Miller's tables, 7 digits).  Independent of the oracle's root
# finding: the roots must round to these.
TEXTBOOK_MU1 = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 10: 0.1893213, 12: 0.1672126}


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12])
def test_mu1_fixed_by_next_even_moment(N):
    """mu_1 is defined by the first even moment the weights are not fitted
    to: sum w Omega_x^N = 4 pi/(N+1) on the sphere.  It holds to rounding,
    and the root agrees with the 7-digit textbook table (a typo or a 1 %
    change of mu_1 fails both)."""
    om, w = Q.level_symmetric(N, 3)
    for i in range(3):
        assert abs(np.dot(w, om[:, i] ** N) - 4 * math.pi / (N + 1)) < 1e-13
    mu1 = np.abs(om).min()
    assert abs(mu1 - TEXTBOOK_MU1[N]) <= 1.5e-7
    # the moment after it is not matched (the set is not a product rule)
    assert abs(np.dot(w, om[:, 0] ** (N + 2)) - 4 * math.pi / (N + 3)) > 1e-6


@pytest.mark.parametrize("N", [4, 8, 12])
def test_perturbed_mu1_breaks_next_moment(N):
    """A 1e-6 relative change of mu_1 violates the defining condition by far
    more than rounding (the condition is a sharp pin on mu_1)."""
    mu1 = Q.mu1_of(N)
    assert abs(Q.next_moment_defect(N, mu1)) < 1e-15
    assert abs(Q.next_moment_defect(N, mu1 * (1 + 1e-6))) > 1e-10
