"""The library's host setup (C++) against the oracle, on the CPU: quadrature
and element matrices to rounding, and the integer graph work -- edges,
quantised weights, lagged edges and levels -- bit for bit."""
import numpy as np
import pytest

import workloads as W
from tests.lib_helpers import graph_parity, rel_err

CASES = {
    "c1": W.c1,
    "cyclic2d": lambda: W.small(dim=2, n=12, r=3, p=2, N=8, amp=0.3 / 12, freq=3),
    "c2crop": lambda: W.make_problem("c2crop", 2, (32, 32), 3, 3, 8, 0.3 / 32, 8, 1.0, 0.8, 1.0),
    "warp3d": lambda: W.small(dim=3, n=4, r=2, p=2, N=4, amp=0.08, freq=1),
    "ragged3d": lambda: W.make_problem("r3", 3, (5, 3, 2), 2, 1, 2, 0.06, 1, 1.0, 0.5, 1.0),
    # strongly warped meshes of the weighting study: cycles of up to 10
    # elements at S2 (exact cut), up to 16 at S8 (Eades-Lin-Smyth)
    "standin2d": lambda: W.standin_2d(16, 21),
    "standin3d": lambda: W.standin_3d(p=1),
    "strongcyc": lambda: W.cyclic_2d(16, 2, 0.9, 1, 8),
    # curved domain boundary: quarter annulus, cycles of up to 9 elements
    "annulus": lambda: W.annulus_quarter(9, 15, 3, 4),
    # unstructured element lists (renumbered, every element's frame rotated
    # at random): a full annulus that closes on itself, a five-block O-grid
    # disk, a cylindrical shell with all 24 rotations of the cube, and
    # lattice meshes given as element lists (cyclic 2D Q3, warped 3D Q2)
    "u_annulus": lambda: W.annulus_full(nr=4, nt=16, p=2, sn_order=4),
    "u_disk": lambda: W.disk_ogrid(n=3, m=2, p=2, sn_order=4),
    "u_shell": lambda: W.annulus_shell_3d(nr=2, nt=8, nz=2, p=2, sn_order=4),
    "u_cyclic2d": lambda: W.as_unstructured(W.small(dim=2, n=12, r=3, p=2, N=8, amp=0.3 / 12, freq=3), 11),
    "u_warp3d": lambda: W.as_unstructured(W.small(dim=3, n=4, r=2, p=2, N=4, amp=0.08, freq=1), 12),
    # curved triangles (renumbered, every element's vertex order turned at
    # random): a warped square, a closed annulus with sign changes of
    # Omega . n and cycles, both at several orders
    "t_square": lambda: W.tri_square(n=6, r=2, p=2, sn_order=4),
    "t_square_q1p1": lambda: W.tri_square(n=8, r=1, p=1, sn_order=8),
    "t_annulus": lambda: W.tri_annulus(nr=3, nt=16, r=3, p=2, sn_order=4),
    "t_annulus_p3": lambda: W.tri_annulus(nr=2, nt=12, r=2, p=3, sn_order=8),
    # curved tetrahedra (renumbered, vertex orders permuted at random): a
    # warped cube cut into Kuhn tetrahedra, a closed cylindrical shell
    "k_cube": lambda: W.tet_cube(n=3, r=2, p=2, sn_order=4),
    "k_cube_p3": lambda: W.tet_cube(n=2, r=1, p=3, sn_order=2),
    "k_shell": lambda: W.tet_shell(nr=2, nt=8, nz=2, r=2, p=1, sn_order=4),
}


@pytest.fixture(scope="module")
def ctx():
    from paper_1810_11080_amd import Context
    return Context(device=-1)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("weighting", [0, 1, 2])
def test_graph_bit_exact(ctx, case, weighting):
    from paper_1810_11080_amd import Problem
    wp = CASES[case]()
    P = Problem.from_workload(ctx, wp, weighting=weighting)
    bad, disc = graph_parity(P, wp, weighting=weighting)
    assert bad == []
    om, w = P.quadrature()
    assert rel_err(om, disc.omega) < 1e-14 and rel_err(w, disc.w) < 1e-13
    M, K = P.element_matrices()
    assert rel_err(M, disc.M) < 1e-13 and rel_err(K, disc.K) < 1e-13


@pytest.mark.parametrize("seed", range(6))
def test_random_problems(ctx, seed):
    from paper_1810_11080_amd import Problem
    wp = W.random_problem(seed, dim=2 if seed % 2 == 0 else 3)
    P = Problem.from_workload(ctx, wp)
    bad, _ = graph_parity(P, wp)
    assert bad == []


def test_exact_limit_one_uses_heuristic(ctx):
    """exact_scc_max = 1 sends every component through Eades-Lin-Smyth."""
    from paper_1810_11080_amd import Problem
    wp = CASES["cyclic2d"]()
    wp.exact_scc_max = 1
    P = Problem.from_workload(ctx, wp)
    bad, _ = graph_parity(P, wp)
    assert bad == []


@pytest.mark.slow
def test_c2_full_graph(ctx):
    """Full 128x128 Q3 S8 workload: all 40 directions bit-exact."""
    from paper_1810_11080_amd import Problem
    wp = W.c2()
    P = Problem.from_workload(ctx, wp)
    info = P.info()
    assert info["n_removed_total"] > 0
    bad, _ = graph_parity(P, wp)
    assert bad == []


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12])
def test_library_mu1_fixed_by_next_even_moment(ctx, N):
    """The library's level-symmetric set satisfies the defining condition of
    mu_1, sum w Omega_x^N = 4 pi/(N+1), to rounding, and its smallest cosine
    rounds to the 7-digit textbook value (pinned without the oracle)."""
    import math
    from paper_1810_11080_amd import Problem
    table = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 10: 0.1893213, 12: 0.1672126}
    wp = W.make_problem("q", 3, (2, 2, 2), 1, 1, N, 0.0, 1, 1.0, 0.5, 1.0)
    P = Problem.from_workload(ctx, wp)
    om, w = P.quadrature()
    for i in range(3):
        assert abs(np.dot(w, om[:, i] ** N) - 4 * math.pi / (N + 1)) < 1e-13
    assert abs(np.abs(om).min() - table[N]) <= 1.5e-7


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c3", "c5"])
def test_full_size_graphs_sampled_directions(ctx, name):
    """Full-size 3D workloads (32^3 S8, 48^3 S12): for one direction per
    octant, the library's edges, quantised weights, lagged edges and levels
    hash to the oracle's (stored by tests/golden/make_large_sweep_samples.py,
    since the oracle needs minutes here)."""
    import hashlib
    import os
    from paper_1810_11080_amd import Problem
    data = np.load(os.path.join(os.path.dirname(__file__), "golden", f"{name}_sweep_samples.npz"))
    wp = {"c3": W.c3, "c5": W.c5}[name]()
    P = Problem.from_workload(ctx, wp)
    for k, d in enumerate(data["dirs"]):
        up, down, w = P.edges(int(d))
        rd, ru = P.removed_edges(int(d))
        lev = P.levels(int(d))
        h = hashlib.sha256()
        for a in (up, down, w, rd, ru, lev):
            h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
        assert (len(up), len(rd), int(lev.max()) + 1) == tuple(data["graph_counts"][k]), int(d)
        assert h.hexdigest() == str(data["graph_sha256"][k]), int(d)


@pytest.mark.parametrize("dim,r,p", [(2, 3, 2), (2, 2, 3), (3, 2, 2)])
def test_node_coordinates_and_volume_rule(ctx, dim, r, p):
    """The library's DG node positions and error-norm rule against the
    oracle's geometry (mesh map at the Gauss-Lobatto nodes; Gauss points,
    weights times |det J| and basis values with two extra points per axis)."""
    from oracle.geometry import ElementGeometry
    from paper_1810_11080_amd import Problem
    n = 5 if dim == 2 else 3
    wp = W.small(dim=dim, n=n, r=r, p=p, N=4, amp=0.08, freq=1)
    P = Problem.from_workload(ctx, wp)
    xyz = P.node_coordinates()
    g = ElementGeometry(wp.lattice, dim, wp.nx, r, p, extra_points=2)
    assert rel_err(xyz, g.dg_node_positions()) < 1e-14
    x, wd, basis = P.volume_rule(extra=2)
    assert rel_err(x, g.x) < 1e-14
    assert rel_err(wd, g.wq[None, :] * g.detJ) < 1e-13
    assert rel_err(basis, g.U) < 1e-14


@pytest.mark.parametrize("r,p", [(2, 2), (3, 1), (1, 3)])
def test_triangle_node_coordinates_and_volume_rule(ctx, r, p):
    """The same on curved triangles (collapsed Gauss rule)."""
    from oracle.simplex import SimplexGeometry
    from paper_1810_11080_amd import Problem
    wp = W.tri_annulus(nr=2, nt=8, r=r, p=p, sn_order=4)
    P = Problem.from_workload(ctx, wp)
    g = SimplexGeometry(wp.nodes[wp.elem_nodes], r, p, extra_points=2)
    assert rel_err(P.node_coordinates(), g.dg_node_positions()) < 1e-14
    x, wd, basis = P.volume_rule(extra=2)
    assert rel_err(x, g.x) < 1e-14
    assert rel_err(wd, g.wq[None, :] * g.detJ) < 1e-13
    assert rel_err(basis, g.U) < 1e-13


@pytest.mark.parametrize("r,p", [(2, 2), (1, 3), (3, 1)])
def test_tet_node_coordinates_and_volume_rule(ctx, r, p):
    """The same on curved tetrahedra (collapsed Gauss rule)."""
    from oracle.simplex import TetGeometry
    from paper_1810_11080_amd import Problem
    wp = W.tet_shell(nr=1, nt=6, nz=1, r=r, p=p, sn_order=2)
    P = Problem.from_workload(ctx, wp)
    g = TetGeometry(wp.nodes[wp.elem_nodes], r, p, extra_points=2)
    assert rel_err(P.node_coordinates(), g.dg_node_positions()) < 1e-14
    x, wd, basis = P.volume_rule(extra=2)
    assert rel_err(x, g.x) < 1e-14
    assert rel_err(wd, g.wq[None, :] * g.detJ) < 1e-13
    assert rel_err(basis, g.U) < 1e-12


def test_set_source_validation(ctx):
    from paper_1810_11080_amd import Problem
    from paper_1810_11080_amd.binding import SnswError
    wp = W.c1()
    P = Problem.from_workload(ctx, wp)
    qd, tab = W.random_direction_data(wp, P.D, 3)
    P.set_source(qd, bc_kind=2, psi_inc_tab=tab)        # host-only: stored, no device work
    with pytest.raises(SnswError):
        P.set_source(qd, bc_kind=2)                      # tabulated without a table
    with pytest.raises(SnswError):
        P.set_source(qd, bc_kind=7)
    bad = qd.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(SnswError) as info:
        P.set_source(bad)
    assert info.value.code == -3


def test_unstructured_input_errors(ctx):
    """Bad element lists are reported, not swept: an index out of range, a
    face shared by three element slots; triangles only as 2D element lists."""
    from paper_1810_11080_amd import Problem, SnswError
    wp = W.annulus_full(nr=2, nt=8, p=1, sn_order=2)
    en = wp.elem_nodes.copy()
    en[3, 0] = len(wp.nodes)
    with pytest.raises(SnswError) as ei:
        Problem(ctx, dim=2, nx=(wp.n_elements, 1), geom_order=wp.r, dg_order=wp.p, lattice=None, sn_order=2,
                sigma_t=wp.sigma_t, sigma_s=wp.sigma_s, q=wp.q, nodes=wp.nodes, elem_nodes=en)
    assert ei.value.code == -1
    dup = np.concatenate([wp.elem_nodes, wp.elem_nodes[:1]])
    E = len(dup)
    with pytest.raises(SnswError) as ei:
        Problem(ctx, dim=2, nx=(E, 1), geom_order=wp.r, dg_order=wp.p, lattice=None, sn_order=2,
                sigma_t=np.ones(E), sigma_s=np.zeros(E), q=np.ones(E), nodes=wp.nodes, elem_nodes=dup)
    assert ei.value.code == -2
    # element lists sweep on the level schedule unless the persistent one is asked for
    assert Problem.from_workload(ctx, wp).info()["schedule"] == 2
    assert Problem.from_workload(ctx, wp, schedule=1).info()["schedule"] == 1
    # simplices: only as element lists, with (r+1)(r+2)/2 control points per
    # triangle
    tw = W.tri_square(n=2, r=2, p=1, sn_order=2)
    E = tw.n_elements
    with pytest.raises(SnswError) as ei:
        Problem(ctx, dim=2, nx=(E, 1), geom_order=2, dg_order=1, lattice=np.zeros(((2 * E + 1) * 3, 2)), sn_order=2,
                sigma_t=tw.sigma_t, sigma_s=tw.sigma_s, q=tw.q, element=1)
    assert ei.value.code == -1
    with pytest.raises(ValueError):   # 3D simplices need (r+1)(r+2)(r+3)/6 control points
        Problem(ctx, dim=3, nx=(E, 1, 1), geom_order=2, dg_order=1, lattice=None, sn_order=2,
                sigma_t=tw.sigma_t, sigma_s=tw.sigma_s, q=tw.q, nodes=np.zeros((len(tw.nodes), 3)),
                elem_nodes=tw.elem_nodes, element=1)
    with pytest.raises(ValueError):
        Problem(ctx, dim=2, nx=(E, 1), geom_order=2, dg_order=1, lattice=None, sn_order=2,
                sigma_t=tw.sigma_t, sigma_s=tw.sigma_s, q=tw.q, nodes=tw.nodes,
                elem_nodes=tw.elem_nodes[:, :5], element=1)


def test_mixed_precision_schedule_choice(ctx):
    """Mixed precision sweeps persistently where the persistent kernels read
    FP32 inverses (2D lattices, inverses not switched off) and level by level
    elsewhere; asking for the persistent schedule elsewhere is refused
    (SNSW_E_UNSUPPORTED)."""
    from paper_1810_11080_amd import Problem, SnswError
    for p in (1, 2, 3):
        wp = W.small(dim=2, n=4, r=2, p=p, N=2)
        assert Problem.from_workload(ctx, wp, precision=1).info()["schedule"] == 1
        assert Problem.from_workload(ctx, wp, precision=1, schedule=2).info()["schedule"] == 2
        assert Problem.from_workload(ctx, wp, precision=1, cache_inverse=2).info()["schedule"] == 2
        with pytest.raises(SnswError) as ei:
            Problem.from_workload(ctx, wp, precision=1, cache_inverse=2, schedule=1)
        assert ei.value.code == -9
    for wp in (W.small(dim=3, n=2, r=1, p=1, N=2), W.small(dim=3, n=2, r=1, p=2, N=2),
               W.annulus_full(nr=2, nt=8, p=1, sn_order=2)):
        assert Problem.from_workload(ctx, wp, precision=1).info()["schedule"] == 2
        with pytest.raises(SnswError) as ei:
            Problem.from_workload(ctx, wp, precision=1, schedule=1)
        assert ei.value.code == -9
