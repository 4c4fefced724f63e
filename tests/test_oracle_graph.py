"""Pins of the oracle's graph work (section 3): Tarjan SCCs against scipy,
the exact minimum feedback arc set against brute force over all orders, the
Eades-Lin-Smyth heuristic on hand-worked graphs, and the invariants of the
cut graph and its levels."""
import itertools

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import workloads as W
from oracle.discretization import Discretization
from oracle.graph import direction_graph, eades_order, exact_order, tarjan_scc


def partition(labels):
    groups = {}
    for v, c in enumerate(labels):
        groups.setdefault(int(c), set()).add(v)
    return {frozenset(s) for s in groups.values()}


@pytest.mark.parametrize("seed", range(8))
def test_tarjan_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(5, 60))
    m = int(rng.integers(V, 3 * V))
    u = rng.integers(0, V, m)
    v = rng.integers(0, V, m)
    adj = [[] for _ in range(V)]
    for a, b in zip(u, v):
        adj[a].append(int(b))
    ours = tarjan_scc(V, adj)
    mat = csr_matrix((np.ones(m), (u, v)), shape=(V, V))
    _, lab = connected_components(mat, directed=True, connection="strong")
    assert partition(ours) == partition(lab)


def lagged_weight(order, W):
    pos = {v: i for i, v in enumerate(order)}
    s = len(order)
    return sum(W[a][b] for a in range(s) for b in range(s) if W[a][b] and pos[a] > pos[b])


@pytest.mark.parametrize("seed", range(12))
def test_exact_fas_is_optimal(seed):
    rng = np.random.default_rng(100 + seed)
    s = int(rng.integers(2, 8))
    Wm = [[0] * s for _ in range(s)]
    for a in range(s):
        for b in range(s):
            if a != b and rng.random() < 0.5:
                Wm[a][b] = int(rng.integers(1, 20))
    order, cost = exact_order(list(range(s)), Wm)
    brute = min(lagged_weight(list(pm), Wm) for pm in itertools.permutations(range(s)))
    assert cost == brute
    assert lagged_weight(order, Wm) == brute


def test_eades_hand_worked():
    # 2-cycle: lag the lighter edge
    out = [{1: 5}, {0: 3}]
    inn = [{1: 3}, {0: 5}]
    assert eades_order([0, 1], out, inn) == [0, 1]
    # 3-cycle with equal weights: all deltas 0, smallest id first
    out = [{1: 1}, {2: 1}, {0: 1}]
    inn = [{2: 1}, {0: 1}, {1: 1}]
    assert eades_order([0, 1, 2], out, inn) == [0, 1, 2]
    # delta(0)=2, delta(1)=3, delta(2)=-5 -> vertex 1 first, then 2 and 0
    # become sinks in turn (0 -> 2 remains): order 1, 0, 2
    out = [{1: 1, 2: 2}, {0: 1, 2: 4}, {1: 1}]
    inn = [{1: 1}, {0: 1, 2: 1}, {0: 2, 1: 4}]
    assert eades_order([0, 1, 2], out, inn) == [1, 0, 2]


def cut_graph_invariants(disc, g):
    rem = set(zip(g.removed_up.tolist(), g.removed_down.tolist()))
    edges = set(zip(g.up.tolist(), g.down.tolist()))
    assert rem <= edges
    for u, v in rem:
        assert g.comp[u] == g.comp[v]
    kept_in = {v: [] for v in range(disc.E)}
    for u, v in edges - rem:
        assert g.level[u] < g.level[v]
        kept_in[v].append(u)
    for v in range(disc.E):
        if g.level[v] > 0:
            assert max(g.level[u] for u in kept_in[v]) == g.level[v] - 1
        else:
            assert not kept_in[v]


@pytest.mark.parametrize("weighting", [0, 1, 2])
def test_cut_graph_invariants_cyclic(weighting):
    prob = W.small(dim=2, n=12, r=3, p=2, N=8, amp=0.3 / 12, freq=3, weighting=weighting)
    disc = Discretization(prob)
    total_removed = 0
    for d in range(disc.D):
        g = direction_graph(disc, d, weighting, 10)
        cut_graph_invariants(disc, g)
        total_removed += len(g.removed_down)
    assert total_removed > 0


def test_large_scc_heuristic_path():
    """Force the Eades path (exact limit 1) and check the invariants."""
    prob = W.small(dim=2, n=12, r=3, p=2, N=8, amp=0.3 / 12, freq=3)
    disc = Discretization(prob)
    for d in (1, 3, 9):
        g = direction_graph(disc, d, 1, 1)
        cut_graph_invariants(disc, g)


@pytest.mark.parametrize("dim,n", [(2, 5), (3, 3)])
def test_unwarped_levels(dim, n):
    prob = W.small(dim=dim, n=n, r=1, p=1, N=4, amp=0.0)
    disc = Discretization(prob)
    for d in range(disc.D):
        g = direction_graph(disc, d, 1, 10)
        assert len(g.removed_down) == 0
        om = disc.omega[d]
        lev = np.zeros(disc.E, dtype=int)
        for a in range(dim):
            ia = disc.eidx[a]
            lev += np.where(om[a] > 0, ia, n - 1 - ia)
        assert np.array_equal(g.level, lev)


@pytest.mark.parametrize("p", [1, 2])
def test_edge_weights_closed_form_unwarped(p):
    """On an unwarped square mesh every x-face block of direction d is
    |Omega_x| times the same face mass matrix and every y-face block
    |Omega_y| times it, so Face weights are rint(|Omega_a| / max_b |Omega_b|
    * 2^20) for an edge across an axis-a face.  SigInvFace multiplies by the
    same M^{-1} up to the element's 1/sigma_t and the x/y symmetry of the
    square, so its weight is rint((|Omega_a| / sigma_down) / max(...) *
    2^20).  Unity weights are 1."""
    n = 4
    sig = np.linspace(0.5, 3.0, n * n)
    wp = W.make_problem("flat", 2, (n, n), 1, p, 4, 0.0, 1, sig, 0.5, 1.0)
    disc = Discretization(wp)
    for d in range(disc.D):
        om = np.abs(disc.omega[d, :2])
        for weighting in (0, 1, 2):
            g = direction_graph(disc, d, weighting)
            # axis of the shared face: elements differ along x (axis 0) or y
            axis = np.where(np.abs(g.up - g.down) == 1, 0, 1)
            if weighting == 0:
                assert np.all(g.w == 1)
                continue
            raw = om[axis] / (sig[g.down] if weighting == 2 else 1.0)
            expect = np.clip(np.rint(raw / raw.max() * 2 ** 20), 1, 2 ** 20).astype(np.int64)
            assert np.array_equal(g.w, expect), (d, weighting)
