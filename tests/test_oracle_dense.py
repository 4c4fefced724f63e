"""The lagged source iteration converges to the exact discrete solution
(brute-force global solve of eq. matrixFormLinearTransport), also on meshes
whose sweep graphs have cycles and lagged edges; the sweep result does not
depend on the element order; local matrices admit LU without pivoting."""
import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, source_iteration, sweep


def cyclic_problem(p=1, N=4, c=0.5, weighting=1, bc=0):
    return W.small(dim=2, n=8, r=3, p=p, N=N, amp=0.3 / 8, freq=2, sigma_t=1.0, c=c, q=1.0,
                   weighting=weighting, bc_kind=bc, psi_inc=0.8 if bc else 0.0)


@pytest.mark.parametrize("p,weighting,bc", [(1, 0, 0), (1, 1, 1), (1, 2, 0)])
def test_fixed_point_equals_dense(p, weighting, bc):
    disc = Discretization(cyclic_problem(p=p, weighting=weighting, bc=bc))
    gs = build_graphs(disc)
    assert sum(len(g.removed_down) for g in gs) > 0
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-13, max_iters=500)
    phid, psid = dense.solve(disc)
    assert np.abs(phi - phid).max() / np.abs(phid).max() < 1e-11
    assert np.abs(psi - psid).max() / np.abs(psid).max() < 1e-11


def test_dense_3d():
    prob = W.small(dim=3, n=3, r=2, p=1, N=2, amp=0.05, freq=1, sigma_t=2.0, c=0.5, q=1.0,
                   bc_kind=W.ISO_CONST, psi_inc=1.0)
    disc = Discretization(prob)
    gs = build_graphs(disc)
    phi, psi, it, rho = source_iteration(disc, gs, tol=1e-13, max_iters=300)
    phid, psid = dense.solve(disc)
    assert np.abs(phi - phid).max() / np.abs(phid).max() < 1e-11


def random_topological_order(g, rng):
    E = len(g.level)
    rem = set(zip(g.removed_up.tolist(), g.removed_down.tolist()))
    adj = [[] for _ in range(E)]
    indeg = np.zeros(E, dtype=int)
    for u, v in zip(g.up.tolist(), g.down.tolist()):
        if (u, v) not in rem:
            adj[u].append(v)
            indeg[v] += 1
    ready = [v for v in range(E) if indeg[v] == 0]
    order = []
    while ready:
        k = int(rng.integers(len(ready)))
        v = ready.pop(k)
        order.append(v)
        for u in adj[v]:
            indeg[u] -= 1
            if indeg[u] == 0:
                ready.append(u)
    assert len(order) == E
    return order


def test_order_independence():
    disc = Discretization(cyclic_problem(p=2, c=0.7))
    gs = build_graphs(disc)
    rng = np.random.default_rng(5)
    phi0 = rng.uniform(0, 1, (disc.E, disc.n))
    psi0 = rng.uniform(0, 1, (disc.D, disc.E, disc.n))
    psi_a, phi_a = sweep(disc, gs, phi0, psi0)
    orders = [random_topological_order(g, rng) for g in gs]
    psi_b, phi_b = sweep(disc, gs, phi0, psi0, serial_orders=orders)
    assert np.abs(psi_a - psi_b).max() < 1e-13 * np.abs(psi_a).max()


def test_local_matrix_symmetric_part_positive():
    prob = W.small(dim=2, n=8, r=3, p=3, N=8, amp=0.3 / 8, freq=2, sigma_t=0.1, c=0.0)
    disc = Discretization(prob)
    for d in range(0, disc.D, 3):
        A = disc.local_matrix(d, np.arange(disc.E))
        ev = np.linalg.eigvalsh(A + A.transpose(0, 2, 1))
        assert ev.min() > 0
