"""Lagged transport sweep and source iteration (oracle).

One sweep solves, for every direction d, eq. laggedSourceIteration

  [G + F_<= + M_t] psi_{l+1} = q + M_s phi_l / (4 pi) - F_> psi_l

element by element in an order compatible with the cut graph: couplings kept
in the graph read the upwind element's new flux, couplings on removed (lagged)
edges read the flux of the previous sweep psi_l.  Reading: the lagged read is
always psi_l, even when the upwind element has already been updated in the
current sweep, which makes the result independent of the traversal order.
Elements are visited level by level (all elements of one level are
independent, so they are solved together); ``serial_orders`` visits them one
at a time in a caller-given topological order instead.

Source iteration (eq. sourceIteration with the scalar flux of eq.
snScalarFlux, summed in ascending direction order) stops when
max|phi_{l+1} - phi_l| / max|phi_{l+1}| <= tol (reading: the paper monitors
the L-infinity difference of successive iterates).
"""
from __future__ import annotations

import numpy as np

from .graph import direction_graph


def lag_masks(disc, g) -> np.ndarray:
    """(E, ns) bool: slot of element receives its inflow on a lagged edge."""
    mask = np.zeros((disc.E, disc.ns), dtype=bool)
    for dn, up in zip(g.removed_down.tolist(), g.removed_up.tolist()):
        slots = np.nonzero(disc.slot_nbr[dn] == up)[0]
        mask[dn, slots] = True
    return mask


def build_graphs(disc, weighting=None, exact_max=None):
    weighting = disc.prob.weighting if weighting is None else weighting
    exact_max = disc.prob.exact_scc_max if exact_max is None else exact_max
    graphs = []
    for d in range(disc.D):
        g = direction_graph(disc, d, weighting, exact_max)
        g.mask = lag_masks(disc, g)
        graphs.append(g)
    return graphs


def sweep(disc, graphs, phi, psi_old, serial_orders=None, solver=None):
    """One lagged sweep.  Returns (psi_new (D,E,n), phi_new (E,n))."""
    D, E, n = disc.D, disc.E, disc.n
    psi_new = np.zeros((D, E, n))
    solve = solver or (lambda A, b: np.linalg.solve(A, b[..., None])[..., 0])
    for d in range(D):
        g = graphs[d]
        if serial_orders is not None:
            groups = [np.array([e]) for e in serial_orders[d]]
        else:
            groups = [np.nonzero(g.level == k)[0] for k in range(int(g.level.max()) + 1)]
        for elems in groups:
            A = disc.local_matrix(d, elems)
            b = disc.local_rhs(d, elems, phi, psi_new[d], psi_old[d], g.mask[elems])
            psi_new[d, elems] = solve(A, b)
    phi_new = np.zeros((E, n))
    for d in range(D):
        phi_new += disc.w[d] * psi_new[d]
    return psi_new, phi_new


def source_iteration(disc, graphs=None, tol=1e-10, max_iters=1000, phi0=None,
                     psi0=None, history=None):
    """Plain source iteration from phi0 (default 0) and lagged traces psi0
    (default 0).  Returns (phi, psi, iterations, last residual)."""
    graphs = graphs if graphs is not None else build_graphs(disc)
    phi = np.zeros((disc.E, disc.n)) if phi0 is None else phi0.copy()
    psi = np.zeros((disc.D, disc.E, disc.n)) if psi0 is None else psi0.copy()
    rho = np.inf
    it = 0
    for it in range(1, max_iters + 1):
        psi, phi_new = sweep(disc, graphs, phi, psi)
        rho = np.abs(phi_new - phi).max() / max(np.abs(phi_new).max(), 1e-300)
        phi = phi_new
        if history is not None:
            history.append(rho)
        if rho <= tol:
            break
    return phi, psi, it, rho
