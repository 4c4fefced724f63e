"""Brute-force global solve of the discrete S_N system (oracle).

Assembles eq. matrixFormLinearTransport for all directions at once,

  (G^(d) + F^(d) + M_t) psi^(d) - (1/4 pi) M_s sum_d' w_d' psi^(d') = q^(d),

as one dense matrix of size D*E*n and solves it with LAPACK.  This is the
"intractable" simultaneous solve the paper avoids; on tiny meshes it gives the
exact discrete solution that the lagged source iteration must converge to.
"""
from __future__ import annotations

import numpy as np


def assemble(disc):
    D, E, n, dim = disc.D, disc.E, disc.n, disc.dim
    N = D * E * n
    A = np.zeros((N, N))
    rhs = np.zeros(N)

    def blk(d, e):
        return slice((d * E + e) * n, (d * E + e + 1) * n)

    elems = np.arange(E)
    zero_phi = np.zeros((E, n))
    for d in range(D):
        Ad = disc.local_matrix(d, elems)
        bd = disc.volume_source(zero_phi, elems, d)
        for e in range(E):
            A[blk(d, e), blk(d, e)] += Ad[e]
            rhs[blk(d, e)] += bd[e]
        for s in range(disc.ns):
            _, Pin = disc.slot_blocks(d, s, elems)
            for e in range(E):
                tn = disc.slot_trace[e, s]
                nb = disc.slot_nbr[e, s]
                rows = blk(d, e).start + tn
                if nb >= 0:
                    cols = blk(d, nb).start + disc.slot_up_trace[e, s]
                    A[np.ix_(rows, cols)] -= Pin[e]
                elif disc.psi_tab is not None:
                    rhs[rows] += Pin[e] @ disc.psi_tab[disc.dir_index(d)][e, tn]
                elif disc.inflow_fn is not None:
                    rhs[rows] += disc.boundary_load(d, s, np.array([e]))[0]
                else:
                    rhs[rows] += Pin[e] @ np.full(len(tn), disc.psi_inc)
        for dp in range(D):
            for e in range(E):
                A[blk(d, e), blk(dp, e)] -= disc.sigma_s[e] / (4.0 * np.pi) * disc.w[dp] * disc.M[e]
    return A, rhs


def solve(disc):
    """Exact discrete solution: (phi (E,n), psi (D,E,n))."""
    A, rhs = assemble(disc)
    x = np.linalg.solve(A, rhs)
    psi = x.reshape(disc.D, disc.E, disc.n)
    phi = np.einsum("d,den->en", disc.w, psi)
    return phi, psi
