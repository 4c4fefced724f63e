"""Pins of the learned-preconditioner oracle: the convolution against scipy's
correlation, the upsample against explicit loops, the hand-written backward
pass against central finite differences, Adam's first step against its closed
form, and the corrected source iteration against plain source iteration
(same fixed point; a zero network reproduces it exactly)."""
import numpy as np
import pytest
from scipy.signal import correlate

import workloads as W
from oracle import learned as LR
from oracle import net as N
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, source_iteration


@pytest.mark.parametrize("stride", [1, 2])
def test_conv3d_matches_scipy(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 6, 7))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    y = N.conv3d(x, w, b, stride)
    for bi in range(2):
        for o in range(4):
            ref = np.full((5, 6, 7), b[o])
            for i in range(3):
                ref += correlate(x[bi, i], w[o, i], mode="same", method="direct")
            assert np.allclose(y[bi, o], ref[::stride, ::stride, ::stride], atol=1e-12)


def test_upsample_add_loops():
    rng = np.random.default_rng(2)
    low = rng.standard_normal((1, 2, 3, 2, 4))
    skip = rng.standard_normal((1, 2, 5, 4, 7))
    out = N.upsample_add(low, skip)
    for c in range(2):
        for z in range(5):
            for y in range(4):
                for x in range(7):
                    assert out[0, c, z, y, x] == low[0, c, z // 2, y // 2, x // 2] + skip[0, c, z, y, x]


def test_backward_matches_finite_differences():
    widths = (2, 3, 3)
    rng = np.random.default_rng(3)
    theta = N.init_params(widths, seed=4) + 0.05 * rng.standard_normal(N.n_params(widths))
    x = rng.standard_normal((2, 3, 5, 4, 3))
    t = rng.standard_normal((2, 1, 5, 4, 3))

    def loss(th):
        y, _ = N.forward(th, widths, x)
        return N.mse(y, t)[0]

    y, cache = N.forward(theta, widths, x)
    _, dy = N.mse(y, t)
    g = N.backward(theta, widths, cache, dy)
    idx = rng.choice(len(theta), size=60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (loss(theta + e) - loss(theta - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_input_gradient_matches_finite_differences():
    widths = (2, 3, 3)
    rng = np.random.default_rng(8)
    theta = N.init_params(widths, seed=2)
    x = rng.standard_normal((1, 3, 4, 3, 5))
    dy = rng.standard_normal((1, 1, 4, 3, 5))
    _, cache = N.forward(theta, widths, x)
    _, dx = N.backward(theta, widths, cache, dy, return_dx=True)
    h = 1e-7
    for idx in [(0, 0, 0, 0, 0), (0, 1, 2, 1, 3), (0, 2, 3, 2, 4), (0, 0, 1, 1, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (np.sum(dy * N.forward(theta, widths, x + e)[0]) - np.sum(dy * N.forward(theta, widths, x - e)[0])) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, dx[idx])


def test_adam_first_step_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    new, m, v = N.adam_step(theta, g, m, v, 1, lr=0.01)
    # bias-corrected first moments are g and g^2: the step is lr*g/(|g|+eps)
    assert np.allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_param_count_of_default_widths():
    # ~200k parameters for widths (16, 32, 32)
    assert N.n_params((16, 32, 32)) == 27 * 7744 + (16 + 16 + 32 + 32 + 32 + 32 + 32 + 32 + 32 + 16 + 16 + 1)


def test_element_average_constant_and_prolongation():
    wp = W.small(dim=2, n=4, r=2, p=2, N=4, amp=0.05)
    disc = Discretization(wp)
    phi = np.full((disc.E, disc.n), 2.5)
    assert np.allclose(LR.element_average(disc, phi), 2.5, atol=1e-14)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((disc.E, disc.n))
    d = rng.standard_normal(disc.E)
    assert np.allclose(LR.element_average(disc, phi + d[:, None]), LR.element_average(disc, phi) + d,
                       atol=1e-13)


def test_zero_network_is_plain_si():
    wp = W.small(dim=2, n=5, r=2, p=1, N=4, amp=0.05, c=0.9)
    disc = Discretization(wp)
    gs = build_graphs(disc)
    widths = (2, 3, 3)
    zero = np.zeros(N.n_params(widths))
    phi_l, hist_l, ncorr = LR.preconditioned_si(disc, gs, zero, widths, 1e-10, 500)
    hist_p = []
    phi_p = source_iteration(disc, gs, tol=1e-10, max_iters=500, history=hist_p)[0]
    assert ncorr > 0
    assert np.array_equal(np.array(hist_l), np.array(hist_p))
    assert np.array_equal(phi_l, phi_p)


def test_random_network_keeps_fixed_point():
    wp = W.small(dim=2, n=5, r=2, p=1, N=4, amp=0.05, c=0.9)
    disc = Discretization(wp)
    gs = build_graphs(disc)
    widths = (2, 3, 3)
    theta = N.init_params(widths, seed=9)
    phi_l, hist_l, _ = LR.preconditioned_si(disc, gs, theta, widths, 1e-12, 2000)
    phi_p = source_iteration(disc, gs, tol=1e-12, max_iters=2000)[0]
    assert hist_l[-1] <= 1e-12
    assert np.abs(phi_l - phi_p).max() / np.abs(phi_p).max() < 1e-9


def test_damping_network_is_linear():
    from tests.lib_helpers import damping_params
    widths = (2, 3, 2)
    th = damping_params(widths, -0.5)
    x = np.random.default_rng(0).uniform(-1, 1, (1, 3, 3, 5, 6))
    y, _ = N.forward(th, widths, x)
    assert np.abs(y[0, 0] + 0.5 * x[0, 0]).max() < 1e-15


@pytest.mark.parametrize("every", [1, 2, 3])
def test_safeguard_rejects_slower_correction(every):
    """A correction that lowers the residual but converges more slowly than
    plain sweeps (under-relaxation by one half) is rejected three times and
    then switched off, for every period including 1 (whose reference plain
    window spans sweeps 1..2): the solve takes at most 3 sweeps more than
    plain source iteration and reaches its fixed point."""
    from tests.lib_helpers import damping_params
    widths = (2, 2, 2)
    wp = W.make_problem("damp", 2, (6, 6), 2, 1, 4, 0.05, 1, 1.0, 0.9, 1.0)
    disc = Discretization(wp)
    gs = build_graphs(disc)
    phi, _, plain_its, _ = source_iteration(disc, gs, tol=1e-10, max_iters=2000)
    phi_c, hist, ncorr = LR.preconditioned_si(disc, gs, damping_params(widths, -0.5), widths, 1e-10, 2000,
                                              every=every)
    assert ncorr == LR.MAX_REJECTIONS
    assert len(hist) <= plain_its + 3
    assert np.abs(phi_c - phi).max() <= 1e-9 * np.abs(phi).max()
