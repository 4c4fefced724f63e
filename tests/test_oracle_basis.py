"""Pins of the oracle's 1D rules and Lagrange bases."""
import math

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_gauss_exactness(n):
    x, w = basis.gauss_legendre(n)
    for k in range(2 * n):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14


def test_gll_closed_forms():
    assert np.allclose(basis.gll_points(1), [0, 1])
    assert np.allclose(basis.gll_points(2), [0, 0.5, 1])
    s = 1 / math.sqrt(5)
    assert np.allclose(basis.gll_points(3), [0, (1 - s) / 2, (1 + s) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange(p):
    nodes = basis.gll_points(p)
    V, D = basis.lagrange(nodes, nodes)
    assert np.allclose(V, np.eye(p + 1), atol=1e-14)
    x = np.linspace(-0.2, 1.3, 17)
    V, D = basis.lagrange(nodes, x)
    assert np.allclose(V.sum(axis=1), 1.0)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-12)
    for k in range(p + 1):
        assert np.allclose(V @ nodes ** k, x ** k, atol=1e-12)
        assert np.allclose(D @ nodes ** k, k * x ** max(k - 1, 0) if k else 0.0, atol=1e-11)
