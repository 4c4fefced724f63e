"""Pins of the oracle on unstructured conforming meshes (element control-point
lists, faces found by matching their corner control points, neighbours that
meet through any pair of slots and any face orientation; section 2's mesh
representation, where each element carries its own control points).

* The same mesh given as a renumbered, locally rotated element list gives the
  same discrete solution as the lattice form (after undoing the renumbering
  and rotations): one lagged sweep on acyclic graphs, the converged source
  iteration (whose fixed point does not depend on the cut) on cyclic ones.
* Genuinely unstructured meshes (a full annulus, which closes on itself; a
  disk whose five-block O-grid has vertices shared by three elements; a
  cylindrical shell whose elements are turned by any of the 24 rotations of
  the cube) reproduce an exact constant solution and agree with the
  brute-force global solve.
The integration-by-parts identity on rotated element lists is in
test_oracle_geometry.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, source_iteration, sweep


def to_unstructured_dofs(u, arr, p):
    """Values per element [..., E, n] of the lattice form, in the element
    numbering and local node order of its unstructured form u."""
    perm, rot = u.meta["perm"], u.meta["rot"]
    maps = [W.local_index_map(u.dim, p + 1, R) for R in W.rotations(u.dim)]
    return np.stack([arr[..., perm[k], :][..., maps[rot[k]]] for k in range(len(perm))], axis=-2)


@pytest.mark.parametrize("prob,seed", [
    (W.c1(), 1),
    (W.small(dim=2, n=(5, 4), r=3, p=3, N=4, amp=0.02, freq=1), 2),
    (W.small(dim=3, n=3, r=2, p=2, N=4, amp=0.05, freq=1, c=0.7), 3),
    (W.small(dim=3, n=(3, 2, 2), r=1, p=1, N=2, amp=0.03, freq=1, bc_kind=W.ISO_CONST, psi_inc=0.5), 4),
], ids=["c1", "2d-q3p3", "3d-q2p2", "3d-q1p1-inflow"])
def test_element_list_form_equals_lattice(prob, seed):
    u = W.as_unstructured(prob, seed=seed)
    d0, d1 = Discretization(prob), Discretization(u)
    g0, g1 = build_graphs(d0), build_graphs(d1)
    perm = u.meta["perm"]
    for a, b in zip(g0, g1):
        # the same edges; and the same cut (these meshes have at most small
        # cycles whose face weights have no ties), so the same levels
        assert set(zip(a.up.tolist(), a.down.tolist())) == \
            set((int(perm[x]), int(perm[y])) for x, y in zip(b.up, b.down))
        assert set(zip(a.removed_down.tolist(), a.removed_up.tolist())) == \
            set((int(perm[x]), int(perm[y])) for x, y in zip(b.removed_down, b.removed_up))
        assert np.array_equal(a.level[perm], b.level)
    rng = np.random.default_rng(7)
    phi0 = rng.uniform(0, 1, (d0.E, d0.n))
    psi0 = rng.uniform(0, 0.2, (d0.D, d0.E, d0.n))
    psi_a, _ = sweep(d0, g0, phi0, psi0)
    psi_b, _ = sweep(d1, g1, to_unstructured_dofs(u, phi0, prob.p), to_unstructured_dofs(u, psi0, prob.p))
    ref = to_unstructured_dofs(u, psi_a, prob.p)
    assert np.abs(psi_b - ref).max() <= 1e-12 * np.abs(ref).max()


def test_element_list_form_cyclic_fixed_point():
    """On a mesh with cycles the cut (and so each iterate) depends on the
    element numbering through the tie-breaks, the converged solution does
    not."""
    prob = W.small(dim=2, n=8, r=3, p=1, N=4, amp=0.3 / 8, freq=2, sigma_t=1.0, c=0.5, q=1.0)
    u = W.as_unstructured(prob, seed=9)
    d0, d1 = Discretization(prob), Discretization(u)
    g0, g1 = build_graphs(d0), build_graphs(d1)
    assert sum(len(g.removed_down) for g in g0) > 0
    phi_a, psi_a, *_ = source_iteration(d0, g0, tol=1e-13, max_iters=500)
    phi_b, psi_b, *_ = source_iteration(d1, g1, tol=1e-13, max_iters=500)
    ref = to_unstructured_dofs(u, psi_a, prob.p)
    assert np.abs(psi_b - ref).max() <= 1e-10 * np.abs(ref).max()


MESHES = {
    "annulus": lambda: W.annulus_full(nr=2, nt=8, p=2, sn_order=4),
    "disk": lambda: W.disk_ogrid(n=2, m=1, p=2, sn_order=4),
    "shell": lambda: W.annulus_shell_3d(nr=1, nt=6, nz=1, p=1, sn_order=2),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_constant_solution_on_unstructured_meshes(name):
    """psi = C solves the transport problem with q = (sigma_t - sigma_s) C
    and inflow C; the DG discretisation reproduces constants, so the
    converged lagged source iteration returns C on every node."""
    from dataclasses import replace
    wp = MESHES[name]()
    C0 = 0.7
    wp = replace(wp, q=(wp.sigma_t - wp.sigma_s) * C0, bc_kind=W.ISO_CONST, psi_inc=C0)
    disc = Discretization(wp)
    assert disc.faces.interior.sum() > 0
    # every interior face is met by two different elements
    assert np.all(disc.faces.minus[disc.faces.interior] != disc.faces.plus[disc.faces.interior])
    phi, psi, *_ = source_iteration(disc, build_graphs(disc), tol=1e-14, max_iters=400)
    assert np.abs(psi - C0).max() < 1e-11


@pytest.mark.parametrize("name", sorted(MESHES))
def test_unstructured_fixed_point_equals_dense(name):
    disc = Discretization(MESHES[name]())
    gs = build_graphs(disc)
    phi, psi, *_ = source_iteration(disc, gs, tol=1e-13, max_iters=400)
    phid, psid = dense.solve(disc)
    assert np.abs(psi - psid).max() / np.abs(psid).max() < 1e-10


def test_annulus_has_cycles_and_closes():
    """The full annulus closes on itself: every element has its neighbours
    across all four slots but the two boundary circles, and sweeps around
    the hole make cycles that are cut."""
    wp = W.annulus_full(nr=2, nt=8, p=1, sn_order=4)
    disc = Discretization(wp)
    assert np.sum(disc.slot_nbr < 0) == 2 * 8       # inner and outer circle only
    gs = build_graphs(disc)
    assert sum(len(g.removed_down) for g in gs) > 0
