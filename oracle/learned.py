"""Source iteration with a learned correction (oracle, NumPy FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Not in the paper (it leaves the strongly scattering regime open); this is
the project's definition, stated plainly:

* element average  a_e(phi) = (1^T M_e phi_e) / (1^T M_e 1), the mean of the
  DG function over element e (M_e the element mass matrix, eq. localMtMatrix
  with sigma = 1);
* after the plain sweep phi~ = S(phi_l) (eq. laggedSourceIteration + eq.
  snScalarFlux), the residual r = phi~ - phi_l gives rbar = a(r) on the
  element grid; s = max |rbar|; the network sees x = [rbar / s,
  log(sigma_t) / 5, c] and its output y gives the correction
  phi_{l+1} = phi~ + s * y_e on every node of element e (a constant per
  element is represented exactly by equal nodal values);
* the plain-sweep residual rho_l = max|phi~ - phi_l| / max|phi~| alone
  decides convergence, so the fixed point is that of plain source iteration;
* the correction is tried after sweeps k, 2k, 3k, ... (k = ``every``), so
  that the plain sweeps in between damp the fast error modes it excites;
* safeguard: the correction is judged over the window of k sweeps that
  follows it, against the plain iteration it replaces -- the mean residual
  reduction per sweep over that window, (rho_t / rho_{t-k})^(1/k), must be
  below the one measured over the latest window without a correction (the
  first window, sweeps 1..k, is plain; a window must span at least one sweep
  to give a rate, so with k = 1 the first correction follows sweep 2);
  otherwise it counts as rejected and the next window is plain.  After 3
  rejections the network is switched off for the rest of the solve.

Training pairs from a plain source iteration converged to phi*: input
x^l = [a(phi_{l+1} - phi_l) / s_l, features], target
t^l = a(phi* - phi_{l+1}) / s_l.
"""
from __future__ import annotations

import numpy as np

from . import net as N
from .sweep import sweep

MAX_REJECTIONS = 3


def element_average(disc, phi):
    """(E,) element means of a DG field phi (E, n)."""
    num = np.einsum("emn,en->e", disc.M, phi)
    den = np.einsum("emn->e", disc.M)
    return num / den


def grid_shape(disc):
    """(Z, Y, X) element grid (Z = 1 in 2D); element e = i + nx (j + ny k)."""
    nx = list(disc.prob.nx) + [1] * (3 - disc.dim)
    return (nx[2], nx[1], nx[0])


def features(disc):
    """(2, Z, Y, X): log(sigma_t)/5 and the scattering ratio c."""
    Z, Y, X = grid_shape(disc)
    st = disc.sigma_t
    c = disc.sigma_s / st
    return np.stack([np.log(st) / 5.0, c]).reshape(2, Z, Y, X)


def make_input(disc, rbar):
    """(1, 3, Z, Y, X) network input and the scale s for residual rbar (E,)."""
    s = float(np.abs(rbar).max())
    Z, Y, X = grid_shape(disc)
    x0 = (rbar / s if s > 0 else np.zeros_like(rbar)).reshape(1, Z, Y, X)
    return np.concatenate([x0, features(disc)])[None], s


def correction(disc, theta, widths, phi_prev, phi_swept):
    """phi~ + s * N(x) prolonged; returns the corrected field (E, n)."""
    rbar = element_average(disc, phi_swept - phi_prev)
    x, s = make_input(disc, rbar)
    if s == 0.0:
        return phi_swept.copy()
    y, _ = N.forward(theta, widths, x)
    return phi_swept + s * y.reshape(-1)[:, None]


def training_pair(disc, phi_prev, phi_swept, phi_star):
    """(x, t) for one plain iteration; x (3, Z, Y, X), t (1, Z, Y, X)."""
    rbar = element_average(disc, phi_swept - phi_prev)
    x, s = make_input(disc, rbar)
    ebar = element_average(disc, phi_star - phi_swept)
    Z, Y, X = grid_shape(disc)
    t = (ebar / s if s > 0 else np.zeros_like(ebar)).reshape(1, Z, Y, X)
    return x[0], t


def preconditioned_si(disc, graphs, theta, widths, tol, max_iters, every=1):
    """Source iteration with the learned correction and the safeguard.
    Returns phi, the residual history and the number of corrected steps."""
    phi = np.zeros((disc.E, disc.n))
    psi = np.zeros((disc.D, disc.E, disc.n))
    hist = []
    enabled, rejections, n_corr = theta is not None, 0, 0
    pending = False                 # the window now ending followed a correction
    start_it, start_res = 1, None   # start of the current window
    plain_rate = np.inf             # per-sweep reduction of the latest plain window
    for it in range(1, max_iters + 1):
        psi, phi_t = sweep(disc, graphs, phi, psi)
        res = float(np.abs(phi_t - phi).max() / np.abs(phi_t).max())
        hist.append(res)
        if res <= tol:
            return phi_t, hist, n_corr
        if start_res is None:
            start_res = res
        apply = False
        if enabled and it % every == 0 and it > start_it:
            rate = (res / start_res) ** (1.0 / max(1, it - start_it))
            apply = True
            if pending:
                if rate >= plain_rate:
                    rejections += 1
                    apply = False
                    if rejections >= MAX_REJECTIONS:
                        enabled = False
            else:
                plain_rate = rate
            pending = apply
            start_it, start_res = it, res
        if apply:
            phi = correction(disc, theta, widths, phi, phi_t)
            n_corr += 1
        else:
            phi = phi_t
    return phi, hist, n_corr
