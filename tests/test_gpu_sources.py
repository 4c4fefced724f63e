"""Direction-dependent sources and tabulated boundary inflow through the
C-ABI (the load vector of eq. qVectorDef from nodal values), against the CPU
FP64 oracle, and the manufactured solution of eq. psiAnnularMMS solved by the
library.

Parity bar as for the other FP64 sweeps: relative L-infinity <= 1e-10.  The
manufactured-solution test compares with the closed form only (no oracle):
the scalar-flux L2 error on warped squares must fall at about order p+1.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.lib_helpers import rel_err
from tests.test_gpu_parity import gpu_sweeps, oracle_sweeps

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_1810_11080_amd import Context
    return Context(device=0)


CASES = {
    # curved 2D mesh with re-entrant faces (some on the boundary), p = 3 and 2
    "cyclic2d_p3": lambda: W.make_problem("cyc_p3", 2, (9, 7), 3, 3, 8, 0.3 / 9, 3, 1.0, 0.7, 1.0),
    "cyclic2d_p2": lambda: W.make_problem("cyc_p2", 2, (10, 6), 3, 2, 6, 0.3 / 10, 3, 1.0, 0.6, 1.0),
    "warp3d_p2": lambda: W.make_problem("w3p2", 3, (4, 3, 3), 2, 2, 4, 0.07, 1, 2.0, 0.5, 1.0),
    "warp3d_p1": lambda: W.make_problem("w3p1", 3, (5, 4, 3), 2, 1, 2, 0.08, 1, 1.0, 0.5, 1.0),
}


def with_direction_data(wp, seed=5):
    D = wp.n_dirs
    qd, tab = W.random_direction_data(wp, D, seed)
    return dataclasses.replace(wp, q_dir=qd, psi_inc_tab=tab, bc_kind=W.TABULATED)


@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "levels"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_direction_source_and_tabulated_inflow(torch, ctx, case, schedule, cache):
    """Seeded nodal source per direction and incident flux per direction and
    boundary node: three sweeps against the oracle, every sweep kernel."""
    from paper_1810_11080_amd import Problem
    wp = with_direction_data(CASES[case]())
    print(f"sources: {case} schedule {schedule} cache {cache}", flush=True)
    P = Problem.from_workload(ctx, wp, schedule=schedule, cache_inverse=cache)
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL
    P.close()


def test_set_source_equals_fresh_problem(torch, ctx):
    """Replacing the source and the boundary condition of a built problem
    gives the sweeps of a problem created with them, bit for bit; switching
    back to the isotropic source restores the original sweeps."""
    from paper_1810_11080_amd import Problem
    base = CASES["cyclic2d_p3"]()
    wp = with_direction_data(base, seed=9)
    P = Problem.from_workload(ctx, base)
    a_phi, _ = gpu_sweeps(torch, P, 2)
    P.reset()
    P.set_source(wp.q_dir, bc_kind=W.TABULATED, psi_inc_tab=wp.psi_inc_tab)
    b_phi, b_psi = gpu_sweeps(torch, P, 2)
    Q = Problem.from_workload(ctx, wp)
    c_phi, c_psi = gpu_sweeps(torch, Q, 2)
    for x, y in zip(b_phi, c_phi):
        assert np.array_equal(x, y)
    assert np.array_equal(b_psi[-1], c_psi[-1])
    P.reset()
    P.set_source(base.q, bc_kind=base.bc_kind, psi_inc=base.psi_inc)
    d_phi, _ = gpu_sweeps(torch, P, 2)
    for x, y in zip(a_phi, d_phi):
        assert np.array_equal(x, y)


def mms_l2_error(torch, ctx, n, p, r=2, amp_cells=0.25, schedule=0):
    """Scalar-flux L2 error of the library's converged solution of the
    manufactured problem on an n x n warped Q_r mesh, S4, sigma_t = 1,
    c = 0.5, incident flux = the exact solution on inflow boundaries."""
    from paper_1810_11080_amd import Problem
    st, ss = 1.0, 0.5
    wp = W.make_problem("mms", 2, (n, n), r, p, 4, amp_cells / n, 1, st, ss / st, 0.0)
    P = Problem.from_workload(ctx, wp, schedule=schedule)
    om, w = P.quadrature()
    xyz = P.node_coordinates()
    q, psi_exact, _ = W.mms_annular(xyz, om, w, st, ss)
    P.set_source(q, bc_kind=W.TABULATED, psi_inc_tab=psi_exact)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    rep = P.solve(phi, tol=1e-13, max_iters=500)
    assert rep["residual"] <= 1e-13
    x, wd, basis = P.volume_rule(extra=4)
    _, _, phi_exact = W.mms_annular(x, om, w, st, ss)
    ph = phi.cpu().numpy().reshape(P.E, P.n) @ basis.T          # (E, Q)
    return float(np.sqrt(np.sum(wd * (ph - phi_exact) ** 2)))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mms_convergence_through_library(torch, ctx, p):
    """eq. psiAnnularMMS on warped squares, S4: the library's scalar flux
    converges at about order p+1 in L2 (upwind DG: between p+1/2 and p+1)."""
    ns = [4, 8, 16]
    errs = [mms_l2_error(torch, ctx, n, p) for n in ns]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    print(f"p={p}: errors {errs}, rates {rates}", flush=True)
    assert rates[-1] > p + 0.4, (errs, rates)


def test_high_order_beats_straightened(torch, ctx):
    """The paper's high-order vs low-order comparison on the quarter annulus
    (curved boundaries, three material rings), manufactured solution,
    S4: the cubic solution on the Q3 mesh is more accurate than the linear
    solution on its straightening (N_ref = 3), with fewer unknowns, and
    refining either mesh lowers its error at about its order (cubic ~ 4,
    linear ~ 2)."""
    import bench
    from paper_1810_11080_amd import Context
    c = Context(0)
    res = {}
    for k in (1, 2):
        ho = W.annulus_quarter(9 * k, 15 * k, 3, 4)
        res[("ho", k)] = bench.mms_error(c, ho)
        res[("lo", k)] = bench.mms_error(c, W.straightened(ho, p=1))
    print({key: (v[0], v[1]) for key, v in res.items()}, flush=True)
    for k in (1, 2):
        assert res[("ho", k)][0] < 0.1 * res[("lo", k)][0]
        assert res[("ho", k)][1] < res[("lo", k)][1]
    assert np.log2(res[("ho", 1)][0] / res[("ho", 2)][0]) > 3.4
    assert np.log2(res[("lo", 1)][0] / res[("lo", 2)][0]) > 1.6
