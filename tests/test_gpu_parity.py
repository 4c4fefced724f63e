"""GPU sweep (HIP, through the C-ABI) against the CPU FP64 oracle.

Bar (FP64 mode): relative L-infinity error <= 1e-10 on the scalar and angular
fluxes, on the same seeded inputs.  Small cases span several blocks and a
ragged tail; the full 128x128 Q3 S8 workload is compared after one sweep from
seeded scalar and lagged angular fluxes; properties (exact constant
solutions, determinism, checkpoint/resume) are checked at full size.
"""
import numpy as np
import pytest

import workloads as W
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, source_iteration, sweep as oracle_sweep
from tests.lib_helpers import rel_err

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


def state_bytes(wp, psi):
    D, E, n = psi.shape
    hdr = np.array([0x534e535745455031, wp.dim, E, n, D, 0, 0, 0], dtype=np.int64)
    return hdr.tobytes() + np.ascontiguousarray(psi, dtype=np.float64).tobytes()


def gpu_sweeps(torch, P, K, phi0=None):
    E, n, D = P.E, P.n, P.D
    phi = torch.zeros(E * n, dtype=torch.float64, device="cuda") if phi0 is None else \
        torch.tensor(phi0.reshape(-1), dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    psi = torch.empty(D * E * n, dtype=torch.float64, device="cuda")
    phis, psis = [], []
    for _ in range(K):
        P.sweep(phi, out, psi)
        torch.cuda.synchronize()
        phis.append(out.cpu().numpy().reshape(E, n).copy())
        psis.append(psi.cpu().numpy().reshape(D, E, n).copy())
        phi, out = out, phi
    return phis, psis


def oracle_sweeps(wp, K, phi0=None, psi0=None):
    disc = Discretization(wp)
    gs = build_graphs(disc)
    phi = np.zeros((disc.E, disc.n)) if phi0 is None else phi0.copy()
    psi = np.zeros((disc.D, disc.E, disc.n)) if psi0 is None else psi0.copy()
    phis, psis = [], []
    for _ in range(K):
        psi, phi = oracle_sweep(disc, gs, phi, psi)
        phis.append(phi)
        psis.append(psi)
    return phis, psis, disc, gs


SMALL = {
    "c1": W.c1,
    "cyclic2d_p1": lambda: W.small(dim=2, n=12, r=3, p=1, N=8, amp=0.3 / 12, freq=3, c=0.7),
    "cyclic2d_p2": lambda: W.small(dim=2, n=12, r=3, p=2, N=8, amp=0.3 / 12, freq=3, c=0.7,
                                   bc_kind=W.ISO_CONST, psi_inc=0.6),
    "cyclic2d_p3": lambda: W.make_problem("cyc_p3", 2, (17, 11), 3, 3, 8, 0.3 / 17, 4,
                                          np.linspace(0.5, 4, 187), 0.6, 1.0),
    "warp3d_p1": lambda: W.small(dim=3, n=5, r=2, p=1, N=4, amp=0.08, freq=1),
    "warp3d_p2": lambda: W.make_problem("w3p2", 3, (5, 4, 3), 2, 2, 4, 0.07, 1,
                                        np.linspace(0.5, 5, 60), 0.8, 1.0,
                                        bc_kind=W.ISO_CONST, psi_inc=0.3),
    "warp3d_p3": lambda: W.small(dim=3, n=3, r=1, p=3, N=2, amp=0.03, freq=1),
    "single2d": lambda: W.small(dim=2, n=1, r=2, p=3, N=4, amp=0.0),
    "single3d": lambda: W.small(dim=3, n=1, r=1, p=2, N=2, amp=0.0),
    "strip": lambda: W.make_problem("strip", 2, (40, 1), 2, 2, 6, 0.02, 1, 1.0, 0.5, 1.0),
    # strongly warped stand-ins of the weighting study (cycles of up to 10
    # elements, inflow 1, sources varying per element)
    "standin2d": lambda: W.standin_2d(16, 21),
    "standin3d": lambda: W.standin_3d(p=1),
    # curved domain boundary (quarter annulus, three material rings)
    "annulus": lambda: W.annulus_quarter(9, 15, 3, 4),
}


@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "levels"])
@pytest.mark.parametrize("case", sorted(SMALL))
def test_sweeps_match_oracle(torch, ctx, case, schedule, cache):
    """Three sweeps per schedule, with the element inverses cached at setup
    or assembled and factored in every sweep."""
    from paper_1810_11080_amd import Problem
    wp = SMALL[case]()
    P = Problem.from_workload(ctx, wp, schedule=schedule, cache_inverse=cache)
    assert P.info()["cached_inverse"] == (1 if cache == 1 else 0)
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


@pytest.mark.parametrize("seed", range(8))
def test_random_problems(torch, ctx, seed):
    from paper_1810_11080_amd import Problem
    wp = W.random_problem(seed, dim=2 if seed < 5 else 3)
    P = Problem.from_workload(ctx, wp)
    g_phi, g_psi = gpu_sweeps(torch, P, 2)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 2)
    assert rel_err(g_phi[-1], o_phi[-1]) < TOL
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


def test_c1_converged(torch, ctx):
    """Source iteration to 1e-12 on the 8x8 Q2 S4 workload."""
    from paper_1810_11080_amd import Problem
    wp = W.c1()
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    rep = P.solve(phi, tol=1e-12, max_iters=200, history_cap=200)
    disc = Discretization(wp)
    o_phi, _, it, _ = source_iteration(disc, tol=1e-12, max_iters=200)
    assert rep["iterations"] == it
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), o_phi) < TOL
    assert rep["history"][-1] <= 1e-12


@pytest.fixture(scope="module")
def c2_oracle():
    wp = W.c2()
    rng = np.random.default_rng(7)
    E, n, D = wp.n_elements, wp.n_dof, wp.n_dirs
    phi0 = rng.uniform(0.0, 2.0, (E, n))
    psi0 = rng.uniform(0.0, 0.2, (D, E, n))
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 1, phi0, psi0)
    return wp, phi0, psi0, o_phi[0], o_psi[0]


@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "levels"])
def test_c2_full_one_sweep(torch, ctx, c2_oracle, schedule, cache):
    """128x128 Q3 p=3 S8 (cyclic graphs), one sweep from seeded scalar flux
    and seeded lagged angular flux, against the oracle."""
    from paper_1810_11080_amd import Problem
    wp, phi0, psi0, o_phi, o_psi = c2_oracle
    P = Problem.from_workload(ctx, wp, schedule=schedule, cache_inverse=cache)
    assert P.info()["n_removed_total"] > 0
    assert P.info()["tile"] == 2     # persistent sweeps take 2x2 tiles here
    P.state_load(state_bytes(wp, psi0))
    g_phi, g_psi = gpu_sweeps(torch, P, 1, phi0)
    P.synchronize()
    assert rel_err(g_phi[0], o_phi) < TOL
    assert rel_err(g_psi[0], o_psi) < TOL


def test_constant_solution_full_size(torch, ctx):
    """sigma_s = 0, q = sigma_t C, psi_inc = C gives psi = C exactly, on the
    full cyclic 128x128 Q3 mesh (lagged couplings converge)."""
    from paper_1810_11080_amd import Problem
    C0 = 1.25
    base = W.c2()
    E = base.n_elements
    st = np.linspace(0.2, 3.0, E)
    wp = W.make_problem("const", 2, base.nx, 3, 3, 8, 0.3 / 128, 32, st, 0.0, st * C0,
                        bc_kind=W.ISO_CONST, psi_inc=C0)
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    psi = torch.empty(P.D * P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-14, max_iters=50, psi=psi, raise_on_not_converged=False)
    assert float((psi - C0).abs().max()) < 1e-10


def test_constant_solution_c5_size(torch, ctx):
    """The same exact constant solution on the 3D 48^3 Q2 p=2 S12 mesh of the
    large configuration (168 directions, 18.6M pairs, two-material sigma_t
    in {1, 100} of seed 100), in the launch configuration bench.py times
    there (level schedule, cached inverses)."""
    from paper_1810_11080_amd import Problem
    C0 = 0.75
    base = W.c5()
    st = base.sigma_t
    wp = W.make_problem("const3d", 3, base.nx, 2, 2, 12, 0.05, 1, st, 0.0, st * C0,
                        bc_kind=W.ISO_CONST, psi_inc=C0)
    P = Problem.from_workload(ctx, wp)
    assert P.info()["cached_inverse"] == 1 and P.info()["schedule"] == 2
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    psi = torch.empty(P.D * P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-14, max_iters=20, psi=psi, raise_on_not_converged=False)
    assert float((psi - C0).abs().max()) < 1e-10
    assert float((phi - 4.0 * np.pi * C0).abs().max()) < 1e-9
    P.close()


@pytest.mark.parametrize("case,cache,precision", [("cyclic2d_p3", 0, 0), ("standin2d", 0, 0), ("cyclic2d_p2", 2, 0),
                                                  ("warp3d_p2", 1, 0), ("cyclic2d_p3", 0, 1), ("cyclic2d_p2", 0, 1)],
                         ids=["dpp", "lds2d", "assembled2d_p2", "inverse3d_p2", "dpp_mixed", "lds2d_mixed"])
def test_wait_failure_reported_and_recovered(torch, ctx, case, cache, precision):
    """The failure path of a persistent sweep, forced from the host: with a
    bound of zero polls every dependency wait whose value is not there at
    the first poll (or at its re-read) gives up at once, the grid drains and
    snsw_synchronize reports SNSW_E_STATE.  With the default bound back and
    the stored flux reset, sweeps equal those of a fresh problem bit for
    bit.  Cases: the DPP kernel (2D p = 3), the LDS kernel with cached
    inverses (2D p = 2 stand-in), the assembled kernel (2D p = 2, no cache)
    and the 3D kernel with cached inverses (p = 2); the DPP and LDS kernels
    with FP32 inverses (mixed precision)."""
    wait_failure_roundtrip(torch, ctx, SMALL[case](), case, cache, precision)


def wait_failure_roundtrip(torch, ctx, wp, case, cache, precision=0):
    from paper_1810_11080_amd import Problem
    from paper_1810_11080_amd.binding import SnswError
    print(f"wait failure: {case}, cache {cache}, precision {precision}", flush=True)
    P = Problem.from_workload(ctx, wp, schedule=1, cache_inverse=cache, precision=precision)
    with pytest.raises(SnswError):
        P.set_wait_limit(-1)
    P.set_wait_limit(0)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    P.sweep(phi, out)
    with pytest.raises(SnswError) as info:
        P.synchronize()
    assert info.value.code == -10
    P.set_wait_limit(1 << 20)
    P.reset()
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    Q = Problem.from_workload(ctx, wp, schedule=1, cache_inverse=cache, precision=precision)
    r_phi, r_psi = gpu_sweeps(torch, Q, 3)
    Q.synchronize()
    for k in range(3):
        assert np.array_equal(g_phi[k], r_phi[k]) and np.array_equal(g_psi[k], r_psi[k])
    P.close()
    Q.close()


def test_determinism_and_checkpoint(torch, ctx):
    from paper_1810_11080_amd import Problem
    wp = SMALL["cyclic2d_p2"]()
    P = Problem.from_workload(ctx, wp)
    a, _ = gpu_sweeps(torch, P, 4)
    P.reset()
    b, _ = gpu_sweeps(torch, P, 4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # checkpoint after 2 sweeps, resume
    P.reset()
    phi2, _ = gpu_sweeps(torch, P, 2)
    st = P.state_save()
    c, _ = gpu_sweeps(torch, P, 1, phi2[-1])
    P.state_load(st)
    d, _ = gpu_sweeps(torch, P, 1, phi2[-1])
    assert np.array_equal(c[0], d[0])
    assert np.array_equal(c[0], a[2])


def test_solve_reports(torch, ctx):
    from paper_1810_11080_amd import Problem, SnswError
    wp = SMALL["cyclic2d_p1"]()
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    with pytest.raises(SnswError) as ei:
        P.solve(phi, tol=1e-30, max_iters=3)
    assert ei.value.code == -5
    P.reset()
    phi.zero_()
    rep = P.solve(phi, tol=1e-11, max_iters=500, check_every=4, history_cap=500)
    assert rep["residual"] <= 1e-11 and rep["iterations"] % 4 == 0
    disc = Discretization(wp)
    o_phi, *_ = source_iteration(disc, tol=1e-13, max_iters=500)
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), o_phi) < 1e-9


def test_c3_full_sampled_directions(torch, ctx):
    """3D 32^3 Q2 p=2 S8 (80 directions): one sweep from seeded scalar and
    lagged angular fluxes; the angular flux of sampled directions (one per
    octant pair) against the oracle restricted to those directions."""
    from oracle.quadrature import level_symmetric
    from paper_1810_11080_amd import Problem
    wp = W.c3()
    P = Problem.from_workload(ctx, wp)
    assert P.info()["cached_inverse"] == 1
    rng = np.random.default_rng(11)
    phi0 = rng.uniform(0.0, 2.0, (P.E, P.n))
    psi0 = rng.uniform(0.0, 0.2, (P.D, P.E, P.n))
    P.state_load(state_bytes(wp, psi0))
    _, g_psi = gpu_sweeps(torch, P, 1, phi0)
    P.synchronize()
    sel = np.array([0, 25, 46, 79])
    om, w = level_symmetric(wp.sn_order, wp.dim)
    disc = Discretization(wp, omega=om[sel], w=w[sel])
    gs = build_graphs(disc)
    o_psi, _ = oracle_sweep(disc, gs, phi0, psi0[sel])
    assert rel_err(g_psi[0][sel], o_psi) < TOL


MIXED_TOL = 1e-5


@pytest.mark.parametrize("cache", [0, 2], ids=["fp32-inverse", "assembled"])
@pytest.mark.parametrize("case", ["c1", "cyclic2d_p3", "warp3d_p2", "warp3d_p3", "strip"])
def test_mixed_precision_sweeps(torch, ctx, case, cache):
    """Mixed precision against the FP64 oracle: the inverse cached in FP32
    (elements of at most 32 nodes; 3D p = 3 falls back to the assembled
    path), or assembled per sweep with an FP32 factorisation and one FP64
    correction."""
    from paper_1810_11080_amd import Problem
    wp = SMALL[case]()
    P = Problem.from_workload(ctx, wp, precision=1, cache_inverse=cache)
    assert P.info()["cached_inverse"] == (2 if cache == 0 and P.n <= 32 else 0)
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < MIXED_TOL
    assert rel_err(g_psi[-1], o_psi[-1]) < MIXED_TOL


@pytest.mark.parametrize("schedule", [1, 2], ids=["persistent", "levels"])
@pytest.mark.parametrize("case", ["c1", "cyclic2d_p2", "cyclic2d_p3"])
def test_mixed_precision_2d_schedules(torch, ctx, case, schedule):
    """FP32 inverses on both 2D schedules: the persistent kernels (DPP on the
    tiled schedule for p = 1, 3; LDS exchanges for p = 2; FP32 rows in
    registers, FP64 products) and the level kernel."""
    from paper_1810_11080_amd import Problem
    wp = SMALL[case]()
    P = Problem.from_workload(ctx, wp, precision=1, schedule=schedule)
    info = P.info()
    assert info["cached_inverse"] == 2 and info["schedule"] == schedule
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < MIXED_TOL
    assert rel_err(g_psi[-1], o_psi[-1]) < MIXED_TOL


@pytest.mark.parametrize("cache,schedule", [(1, 0), (1, 2), (2, 0)],
                         ids=["fp32-inverse-persistent", "fp32-inverse-levels", "assembled"])
def test_mixed_precision_c2_full(torch, ctx, c2_oracle, cache, schedule):
    from paper_1810_11080_amd import Problem
    wp, phi0, psi0, o_phi, o_psi = c2_oracle
    P = Problem.from_workload(ctx, wp, precision=1, cache_inverse=cache, schedule=schedule)
    info = P.info()
    assert info["cached_inverse"] == (2 if cache == 1 else 0)
    # AUTO: persistent with the FP32 inverses, else level by level
    assert info["schedule"] == (schedule if schedule else (1 if cache == 1 else 2))
    P.state_load(state_bytes(wp, psi0))
    g_phi, g_psi = gpu_sweeps(torch, P, 1, phi0)
    P.synchronize()
    assert rel_err(g_phi[0], o_phi) < MIXED_TOL
    assert rel_err(g_psi[0], o_psi) < MIXED_TOL


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_partial_inverse_cache(torch, ctx, precision):
    """A cache budget below the whole set of inverses (level schedule): the
    first directions that fit keep their inverses, the others are assembled
    in every sweep (two launches per level), against the oracle.  A budget
    below one direction caches nothing; persistent schedules cache all or
    nothing."""
    from paper_1810_11080_amd import Problem
    wp = SMALL["warp3d_p2"]()
    full = Problem.from_workload(ctx, wp, precision=precision)
    info = full.info()
    D, E, blk = full.D, full.E, info["inverse_block_bytes"]
    assert info["cached_dirs"] == D and blk == (8 * 730 if precision == 0 else 4 * 4 * 7 * 27)
    full.close()
    P = Problem.from_workload(ctx, wp, precision=precision, cache_budget=(D // 3 + 0.5) * E * blk)
    info = P.info()
    assert info["cached_dirs"] == D // 3 and info["cached_inverse"] == 1 + precision and info["schedule"] == 2
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    tol = MIXED_TOL if precision else TOL
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < tol
    assert rel_err(g_psi[-1], o_psi[-1]) < tol
    P.close()
    Q = Problem.from_workload(ctx, wp, precision=precision, cache_budget=0.5 * E * blk)
    assert Q.info()["cached_dirs"] == 0 and Q.info()["cached_inverse"] == 0
    Q.close()
    if precision == 0:
        R = Problem.from_workload(ctx, wp, schedule=1, cache_budget=(D // 3 + 0.5) * E * blk)
        assert R.info()["cached_dirs"] == 0
        R.close()


@pytest.mark.parametrize("name,precision,part", [("c3", 0, 0), ("c3", 0, 1), ("c5", 0, 0), ("c5", 1, 0)],
                         ids=["c3", "c3-partial-cache", "c5", "c5-mixed"])
def test_full_size_sampled_directions_stored(torch, ctx, name, precision, part):
    """Full-size 3D workloads in the configuration bench.py times (level
    schedule, cached inverses): 32^3 Q2 p=2 S8 (checkerboard sigma_t in
    {1, 10}, c = 0.9) and 48^3 Q2 p=2 S12 (sigma_t in {1, 100} at random,
    c = 0.99).  One sweep from seeded scalar and lagged angular fluxes
    (scattering source on); the angular flux of one direction per octant on
    sampled elements against the oracle's values, stored by
    tests/golden/make_large_sweep_samples.py (the oracle takes minutes
    here).  Mixed precision (the inverses kept in FP32) at the 1e-5 bar.
    part: a cache budget of half the directions (the sampled ones on both
    sides of the split)."""
    import os
    from paper_1810_11080_amd import Problem
    data = np.load(os.path.join(os.path.dirname(__file__), "golden", f"{name}_sweep_samples.npz"))
    wp = {"c3": W.c3, "c5": W.c5}[name]()
    dirs, elems = data["dirs"], data["elems"]
    print(f"{name}: building problem", flush=True)
    budget = 0.0
    if part:
        from oracle.quadrature import level_symmetric
        E, D = int(np.prod(wp.nx)), len(level_symmetric(wp.sn_order, wp.dim)[1])
        budget = (D // 2 + 0.5) * E * 8 * 730          # FP64 blocks of 3D p = 2: 730 doubles
    P = Problem.from_workload(ctx, wp, precision=precision, cache_budget=budget)
    info = P.info()
    assert info["cached_inverse"] == 1 + precision and info["schedule"] == 2
    assert info["cached_dirs"] == (P.D // 2 if part else P.D)
    if part:
        assert info["inverse_block_bytes"] == 8 * 730 and min(dirs) < P.D // 2 <= max(dirs)
    phi0, psi0 = W.sweep_inputs(wp, int(data["seed"]), dirs)
    # lagged state: the sampled directions seeded, the others zero (directions
    # are independent within a sweep)
    state = np.zeros(8 + P.D * P.E * P.n)
    state[:8].view(np.int64)[:] = [0x534e535745455031, wp.dim, P.E, P.n, P.D, 0, 0, 0]
    body = state[8:].reshape(P.D, P.E, P.n)
    for d in dirs:
        body[d] = psi0[int(d)]
    P.state_load(state)
    del state, body
    print(f"{name}: sweeping", flush=True)
    phi = torch.tensor(phi0.reshape(-1), dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    psi = torch.empty(P.D * P.E * P.n, dtype=torch.float64, device="cuda")
    P.sweep(phi, out, psi)
    P.synchronize()
    dd = torch.tensor(dirs, device="cuda")
    ee = torch.tensor(elems, device="cuda")
    got = psi.view(P.D, P.E, P.n).index_select(0, dd).index_select(1, ee).cpu().numpy()
    ref = data["psi"]
    assert got.shape == ref.shape
    for k, d in enumerate(dirs):
        assert rel_err(got[k], ref[k]) < (MIXED_TOL if precision else TOL), (name, int(d))
    P.close()


UNSTRUCTURED = {
    # a full annulus closing on itself (cycles around the hole), Q3, p = 2
    "u_annulus": lambda: W.annulus_full(nr=4, nt=16, p=2, sn_order=4),
    "u_annulus_p3": lambda: W.annulus_full(nr=3, nt=12, p=3, sn_order=8, seed=5),
    # five-block O-grid disk (vertices shared by three elements), Q2, p = 1 / 2
    "u_disk": lambda: W.disk_ogrid(n=3, m=2, p=2, sn_order=4),
    "u_disk_p1": lambda: W.disk_ogrid(n=4, m=3, p=1, sn_order=6, seed=7),
    # cylindrical shell, elements turned by any of the 24 rotations of the cube
    "u_shell": lambda: W.annulus_shell_3d(nr=2, nt=8, nz=2, p=2, sn_order=4),
    "u_shell_p1": lambda: W.annulus_shell_3d(nr=2, nt=10, nz=3, p=1, sn_order=2, seed=8),
    # lattice meshes given as renumbered, rotated element lists
    "u_c1": lambda: W.as_unstructured(W.c1(), 13),
    "u_cyclic2d_p3": lambda: W.as_unstructured(W.make_problem("cyc_p3", 2, (9, 7), 3, 3, 8, 0.3 / 9, 2,
                                                              np.linspace(0.5, 4, 63), 0.6, 1.0,
                                                              bc_kind=W.ISO_CONST, psi_inc=0.4), 14),
}


@pytest.mark.parametrize("schedule", [2, 1], ids=["levels", "persistent"])
@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("case", sorted(UNSTRUCTURED))
def test_unstructured_sweeps_match_oracle(torch, ctx, case, cache, schedule):
    """Unstructured conforming meshes: three sweeps against the oracle, with
    cached inverses and assembled per sweep, on the level schedule and on the
    generic persistent kernels (per-value waits, upwind nodes from the
    table)."""
    from paper_1810_11080_amd import Problem
    wp = UNSTRUCTURED[case]()
    P = Problem.from_workload(ctx, wp, cache_inverse=cache, schedule=schedule)
    assert P.info()["schedule"] == schedule
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


@pytest.mark.parametrize("case", ["u_annulus", "u_shell"])
def test_unstructured_mixed_and_converged(torch, ctx, case):
    """Mixed precision on unstructured meshes (1e-5), and the converged FP64
    solve against the oracle's converged source iteration."""
    from paper_1810_11080_amd import Problem
    from oracle.sweep import source_iteration
    wp = UNSTRUCTURED[case]()
    Pm = Problem.from_workload(ctx, wp, precision=1)
    g_phi, _ = gpu_sweeps(torch, Pm, 2)
    Pm.synchronize()
    o_phi, _, disc, gs = oracle_sweeps(wp, 2)
    assert rel_err(g_phi[-1], o_phi[-1]) < MIXED_TOL
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-12, max_iters=2000)
    ref, *_ = source_iteration(disc, gs, tol=1e-13, max_iters=2000)
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), ref) < 1e-9


SIMPLEX = {
    # curved P_r triangles, renumbered with turned local frames; G = 21 / 10 /
    # 6 pairs per wavefront for p = 1 / 2 / 3, so levels span several blocks
    # and end in ragged batches
    "t_square_p1": lambda: W.tri_square(n=8, r=1, p=1, sn_order=8),
    "t_square_p2": lambda: W.tri_square(n=10, r=2, p=2, sn_order=4, seed=21),
    "t_square_p3": lambda: W.tri_square(n=5, r=3, p=3, sn_order=4, seed=22),
    # closed annulus: sign changes of Omega . n on curved faces, cycles
    "t_annulus_p2": lambda: W.tri_annulus(nr=4, nt=24, r=2, p=2, sn_order=6, seed=23),
    "t_annulus_p3": lambda: W.tri_annulus(nr=3, nt=16, r=3, p=3, sn_order=4, seed=24),
    # one cell: two triangles
    "t_single": lambda: W.tri_square(n=1, r=2, p=2, sn_order=2, seed=None),
}


@pytest.mark.parametrize("schedule", [2, 1], ids=["levels", "persistent"])
@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("case", sorted(SIMPLEX))
def test_triangle_sweeps_match_oracle(torch, ctx, case, cache, schedule):
    """Triangle meshes: three sweeps against the oracle, with cached inverses
    and assembled per sweep, level schedule and persistent kernels."""
    from paper_1810_11080_amd import Problem
    wp = SIMPLEX[case]()
    P = Problem.from_workload(ctx, wp, cache_inverse=cache, schedule=schedule)
    assert P.info()["schedule"] == schedule and P.n == (wp.p + 1) * (wp.p + 2) // 2
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


@pytest.mark.parametrize("case", ["t_annulus_p2", "t_square_p3"])
def test_triangle_mixed_and_converged(torch, ctx, case):
    """Mixed precision on triangles (1e-5), and the converged FP64 solve
    against the oracle's converged source iteration."""
    from paper_1810_11080_amd import Problem
    wp = SIMPLEX[case]()
    Pm = Problem.from_workload(ctx, wp, precision=1)
    g_phi, _ = gpu_sweeps(torch, Pm, 2)
    Pm.synchronize()
    o_phi, _, disc, gs = oracle_sweeps(wp, 2)
    assert rel_err(g_phi[-1], o_phi[-1]) < MIXED_TOL
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-12, max_iters=2000)
    ref, *_ = source_iteration(disc, gs, tol=1e-13, max_iters=2000)
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), ref) < 1e-9


@pytest.mark.parametrize("r,p", [(2, 2), (3, 3), (2, 3)])
def test_triangle_linear_solution_exact(torch, ctx, r, p):
    """A linear angular flux a_d + b_d . x (in the DG space for r <= p) with
    its manufactured source and tabulated inflow is reproduced exactly by
    the converged GPU solve on curved triangles with sign changes of
    Omega . n (no oracle involved: the exact function is the reference)."""
    from paper_1810_11080_amd import Problem
    wp = W.tri_annulus(nr=3, nt=12, r=r, p=p, sn_order=4, seed=25)
    wp.sigma_s[:] = 0.0
    P0 = Problem.from_workload(ctx, wp)
    xn = P0.node_coordinates()
    om, _ = P0.quadrature()
    rng = np.random.default_rng(12)
    a = rng.uniform(0.5, 1.5, P0.D)
    b = rng.uniform(-0.3, 0.3, (P0.D, 2))
    psi_exact = a[:, None, None] + np.einsum("dc,enc->den", b, xn)
    wp.q_dir = np.einsum("dc,dc->d", om[:, :2], b)[:, None, None] + wp.sigma_t[None, :, None] * psi_exact
    wp.bc_kind = W.TABULATED
    wp.psi_inc_tab = psi_exact
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-13, max_iters=500)
    phi_exact = np.einsum("d,den->en", P.quadrature()[1], psi_exact)
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), phi_exact) < 1e-11


ROMBERG = {
    "quads_q3p2": lambda: W.small(dim=2, n=8, r=3, p=2, N=4, amp=0.3 / 8, freq=2, c=0.7),
    "t_annulus_p3": SIMPLEX["t_annulus_p3"],
}


@pytest.mark.parametrize("case", sorted(ROMBERG))
def test_romberg_face_rule_sweeps(torch, ctx, case):
    """Sign-changing faces integrated by adaptive Romberg (tolerance 1e-12):
    three GPU sweeps against the oracle with its own Romberg face rule
    (the two Romberg implementations agree to the tolerance, far below the
    parity bar)."""
    from dataclasses import replace
    from paper_1810_11080_amd import Problem
    wp = replace(ROMBERG[case](), face_rule="romberg", face_tol=1e-12)
    P = Problem.from_workload(ctx, wp, schedule=2)
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


@pytest.mark.parametrize("case,cache", [("t_annulus_p2", 1), ("t_square_p3", 2), ("u_annulus", 1), ("u_shell", 2)])
def test_wait_failure_element_lists(torch, ctx, case, cache):
    """The forced failure path (zero-poll wait bound) of the generic
    persistent kernels on element lists, and recovery bit for bit."""
    wait_failure_roundtrip(torch, ctx, (SIMPLEX if case in SIMPLEX else UNSTRUCTURED)[case](), case, cache)


TETS = {
    # curved P_r tetrahedra, renumbered with permuted vertex orders; G = 16 /
    # 6 / 3 pairs per wavefront for p = 1 / 2 / 3
    "k_cube_p1": lambda: W.tet_cube(n=2, r=1, p=1, sn_order=4),
    "k_cube_p2": lambda: W.tet_cube(n=3, r=2, p=2, sn_order=2, seed=31),
    "k_cube_p3": lambda: W.tet_cube(n=2, r=1, p=3, sn_order=2, seed=32),
    # closed cylindrical shell: sign changes of Omega . n on curved faces, cycles
    "k_shell_p2": lambda: W.tet_shell(nr=2, nt=8, nz=2, r=2, p=2, sn_order=4, seed=33),
}


@pytest.mark.parametrize("schedule", [2, 1], ids=["levels", "persistent"])
@pytest.mark.parametrize("cache", [1, 2], ids=["inverse", "assembled"])
@pytest.mark.parametrize("case", sorted(TETS))
def test_tet_sweeps_match_oracle(torch, ctx, case, cache, schedule):
    """Tetrahedron meshes: three sweeps against the oracle, with cached
    inverses and assembled per sweep, level schedule and persistent kernels."""
    from paper_1810_11080_amd import Problem
    wp = TETS[case]()
    P = Problem.from_workload(ctx, wp, cache_inverse=cache, schedule=schedule)
    assert P.info()["schedule"] == schedule and P.n == (wp.p + 1) * (wp.p + 2) * (wp.p + 3) // 6
    g_phi, g_psi = gpu_sweeps(torch, P, 3)
    P.synchronize()
    o_phi, o_psi, _, _ = oracle_sweeps(wp, 3)
    for k in range(3):
        assert rel_err(g_phi[k], o_phi[k]) < TOL, (case, k)
    assert rel_err(g_psi[-1], o_psi[-1]) < TOL


@pytest.mark.parametrize("case,cache", [("k_shell_p2", 0), ("k_cube_p3", 2)])
def test_tet_mixed(torch, ctx, case, cache):
    """Mixed precision on tetrahedra (FP32 inverses / assembled), 1e-5."""
    from paper_1810_11080_amd import Problem
    wp = TETS[case]()
    P = Problem.from_workload(ctx, wp, precision=1, cache_inverse=cache)
    g_phi, _ = gpu_sweeps(torch, P, 2)
    P.synchronize()
    o_phi, _, _, _ = oracle_sweeps(wp, 2)
    assert rel_err(g_phi[-1], o_phi[-1]) < MIXED_TOL


@pytest.mark.parametrize("r,p", [(1, 1), (2, 2)])
def test_tet_linear_solution_exact(torch, ctx, r, p):
    """A linear angular flux (r <= p) with its manufactured source and
    tabulated inflow, reproduced by the converged GPU solve on curved
    tetrahedra with sign changes of Omega . n (the exact function is the
    reference)."""
    from paper_1810_11080_amd import Problem
    wp = W.tet_shell(nr=2, nt=8, nz=1, r=r, p=p, sn_order=4, seed=34)
    wp.sigma_s[:] = 0.0
    P0 = Problem.from_workload(ctx, wp)
    xn = P0.node_coordinates()
    om, w = P0.quadrature()
    rng = np.random.default_rng(14)
    a = rng.uniform(0.5, 1.5, P0.D)
    b = rng.uniform(-0.3, 0.3, (P0.D, 3))
    psi_exact = a[:, None, None] + np.einsum("dc,enc->den", b, xn)
    wp.q_dir = np.einsum("dc,dc->d", om, b)[:, None, None] + wp.sigma_t[None, :, None] * psi_exact
    wp.bc_kind = W.TABULATED
    wp.psi_inc_tab = psi_exact
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    P.solve(phi, tol=1e-13, max_iters=500)
    phi_exact = np.einsum("d,den->en", w, psi_exact)
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), phi_exact) < 1e-11


@pytest.mark.parametrize("case,cache", [("k_shell_p2", 1), ("k_cube_p1", 2)])
def test_wait_failure_tets(torch, ctx, case, cache):
    """The forced failure path of the persistent kernels on tetrahedra."""
    wait_failure_roundtrip(torch, ctx, TETS[case](), case, cache)
