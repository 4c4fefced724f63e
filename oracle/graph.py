"""Per-direction sweep graph, cycle cutting and levels (oracle; section 3).

Vertices are elements; for a direction d there is an edge up -> down whenever
the coupling block F_{down,up} is nonzero, i.e. the downwind element receives
inflow from the upwind one through their shared face.  Edge weights (list in
section 3, eq. graphWeight), with ||A|| the maximum-entry norm:
  0 Unity        z = 1
  1 Face         z = ||F_{down,up}||
  2 SigInvFace   z = ||M_{t,down}^{-1} F_{down,up}||
Weights are made integer so that the graph work is exact (reading): Unity is
w = 1; otherwise w = clamp(rint(z / z_max * 2^20), 1, 2^20) with ties to even
and z_max the largest z of the direction.

The ordering problem is the minimum feedback arc set: choose an element order
that minimises the total weight of the couplings whose upwind element comes
*after* the downwind one -- those couplings are lagged (read from the previous
iterate) in the sweep.  (Reading: the printed sum runs over e' < e while the
text calls the lagged, upper-triangular part the forward edges; the quantity
minimised is the lagged weight.)  It is solved independently per strongly
connected component (Tarjan):
* components of at most ``exact_max`` (default 10) vertices exactly, by a
  dynamic programme over vertex subsets (the paper's integer programme; same
  optimum).  Vertices are taken in ascending element id; f(T) is the least
  lagged weight of an order of T, f(T) = min_v [f(T \\ v) + sum_{u in T\\v}
  w(v->u)] with v placed last; ties go to the smallest v.
* larger components with the Eades-Lin-Smyth greedy heuristic (weighted):
  repeatedly peel sinks (smallest id first, prepended to the tail sequence)
  and sources (smallest id first, appended to the head sequence); when
  neither exists append the vertex of largest w_out - w_in (ties: smallest
  id).  The order is head + tail; the lagged set is the backward edges.

Levels (not in the paper, which sweeps in a serial order): ASAP level of each
element in the graph without the lagged edges; elements of one level are
mutually independent.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

QUANT = 1 << 20


@dataclass
class GraphResult:
    up: np.ndarray            # (m,) int, edge up -> down
    down: np.ndarray
    w: np.ndarray             # (m,) int64 quantised weights
    z: np.ndarray             # (m,) float weights before quantisation
    comp: np.ndarray          # (E,) SCC label
    removed_down: np.ndarray  # lagged edges, sorted by (down, up)
    removed_up: np.ndarray
    level: np.ndarray         # (E,) int
    stats: dict = field(default_factory=dict)


# ----------------------------------------------------------------------
def edges_for_direction(disc, d: int, weighting: int):
    """Edges (up, down), raw weights z and quantised weights w."""
    fs = disc.faces
    Pp, Pm, mp, mm = disc.face_blocks(d)[:4]
    ups, downs, zs = [], [], []
    interior = np.nonzero(fs.interior)[0]
    for side_blocks, mask, up_el, down_el, down_side in (
            (Pm, mm > 0.0, fs.plus, fs.minus, 0),   # minus receives from plus
            (Pp, mp > 0.0, fs.minus, fs.plus, 1)):  # plus receives from minus
        f = interior[mask[interior]]
        if len(f) == 0:
            continue
        up, down = up_el[f], down_el[f]
        blocks = side_blocks[f]
        if weighting == 0:
            z = np.ones(len(f))
        elif weighting == 1:
            z = np.abs(blocks).max(axis=(1, 2))
        elif weighting == 2:
            # slot of the downwind element on this face and its nodes there
            slot = disc.face_slot[f, down_side]
            tn = disc.slot_trace[down, slot]                       # (k, nf)
            Mt = disc.sigma_t[down, None, None] * disc.M[down]
            Minv = np.linalg.inv(Mt)
            cols = np.take_along_axis(Minv, tn[:, None, :], axis=2)   # Minv[:, :, tn]
            prod = np.einsum("kma,kab->kmb", cols, blocks)
            z = np.abs(prod).max(axis=(1, 2))
        else:
            raise ValueError("weighting")
        ups.append(up)
        downs.append(down)
        zs.append(z)
    if ups:
        up = np.concatenate(ups)
        down = np.concatenate(downs)
        z = np.concatenate(zs)
    else:
        up = down = np.zeros(0, dtype=np.int64)
        z = np.zeros(0)
    if weighting == 0 or len(z) == 0:
        w = np.ones(len(z), dtype=np.int64)
    else:
        w = np.clip(np.rint(z / z.max() * QUANT), 1, QUANT).astype(np.int64)
    return up.astype(np.int64), down.astype(np.int64), z, w


# ----------------------------------------------------------------------
def tarjan_scc(V: int, adj) -> np.ndarray:
    """Strongly connected components (Tarjan 1972), iterative."""
    index = [-1] * V
    low = [0] * V
    on = [False] * V
    comp = [-1] * V
    stack = []
    counter = 0
    ncomp = 0
    for v0 in range(V):
        if index[v0] != -1:
            continue
        index[v0] = low[v0] = counter
        counter += 1
        stack.append(v0)
        on[v0] = True
        work = [[v0, 0]]
        while work:
            v, i = work[-1]
            if i < len(adj[v]):
                work[-1][1] = i + 1
                u = adj[v][i]
                if index[u] == -1:
                    index[u] = low[u] = counter
                    counter += 1
                    stack.append(u)
                    on[u] = True
                    work.append([u, 0])
                elif on[u]:
                    low[v] = min(low[v], index[u])
            else:
                work.pop()
                if work:
                    parent = work[-1][0]
                    low[parent] = min(low[parent], low[v])
                if low[v] == index[v]:
                    while True:
                        u = stack.pop()
                        on[u] = False
                        comp[u] = ncomp
                        if u == v:
                            break
                    ncomp += 1
    return np.array(comp, dtype=np.int64)


def exact_order(verts, W):
    """Optimal order of a small component; W[i][j] = weight of edge i -> j
    between the local vertices (ascending element id)."""
    s = len(verts)
    full = (1 << s) - 1
    f = [0] * (full + 1)
    best = [-1] * (full + 1)
    for T in range(1, full + 1):
        bv, bc = -1, None
        for v in range(s):
            if not (T >> v) & 1:
                continue
            rest = T & ~(1 << v)
            c = f[rest]
            for u in range(s):
                if (rest >> u) & 1:
                    c += W[v][u]
            if bc is None or c < bc:
                bc, bv = c, v
        f[T] = bc
        best[T] = bv
    order_rev = []
    T = full
    while T:
        v = best[T]
        order_rev.append(v)
        T &= ~(1 << v)
    return order_rev[::-1], f[full]


def eades_order(verts, out_edges, in_edges):
    """Weighted Eades-Lin-Smyth ordering of one component.

    out_edges[v] / in_edges[v]: dict neighbour -> weight (component-internal),
    vertices given by local index (ascending element id)."""
    s = len(verts)
    alive = [True] * s
    outdeg = [len(out_edges[v]) for v in range(s)]
    indeg = [len(in_edges[v]) for v in range(s)]
    wout = [sum(out_edges[v].values()) for v in range(s)]
    win = [sum(in_edges[v].values()) for v in range(s)]
    head, tail = [], []
    left = s

    def remove(v):
        nonlocal left
        alive[v] = False
        left -= 1
        for u, wt in out_edges[v].items():
            if alive[u]:
                indeg[u] -= 1
                win[u] -= wt
        for u, wt in in_edges[v].items():
            if alive[u]:
                outdeg[u] -= 1
                wout[u] -= wt

    while left:
        while True:
            sinks = [v for v in range(s) if alive[v] and outdeg[v] == 0]
            if not sinks:
                break
            v = sinks[0]
            remove(v)
            tail.insert(0, v)
        while True:
            srcs = [v for v in range(s) if alive[v] and indeg[v] == 0]
            if not srcs:
                break
            v = srcs[0]
            remove(v)
            head.append(v)
        if left:
            bv, bd = -1, None
            for v in range(s):
                if alive[v]:
                    dlt = wout[v] - win[v]
                    if bd is None or dlt > bd:
                        bd, bv = dlt, v
            remove(bv)
            head.append(bv)
    return head + tail


def direction_graph(disc, d: int, weighting: int = 1, exact_max: int = 10) -> GraphResult:
    E = disc.E
    up, down, z, w = edges_for_direction(disc, d, weighting)
    adj = [[] for _ in range(E)]
    for u, v in zip(up.tolist(), down.tolist()):
        adj[u].append(v)
    comp = tarjan_scc(E, adj)
    # group component members
    members = {}
    for v in range(E):
        members.setdefault(int(comp[v]), []).append(v)
    edge_w = {}
    for u, v, ww in zip(up.tolist(), down.tolist(), w.tolist()):
        edge_w[(u, v)] = ww
    removed = []
    sizes = []
    for c, verts in members.items():
        if len(verts) < 2:
            continue
        verts = sorted(verts)
        sizes.append(len(verts))
        loc = {v: i for i, v in enumerate(verts)}
        s = len(verts)
        if s <= exact_max:
            W = [[0] * s for _ in range(s)]
            for v in verts:
                for u in adj[v]:
                    if u in loc:
                        W[loc[v]][loc[u]] = edge_w[(v, u)]
            order, _ = exact_order(verts, W)
        else:
            out_e = [dict() for _ in range(s)]
            in_e = [dict() for _ in range(s)]
            for v in verts:
                for u in adj[v]:
                    if u in loc:
                        out_e[loc[v]][loc[u]] = edge_w[(v, u)]
                        in_e[loc[u]][loc[v]] = edge_w[(v, u)]
            order = eades_order(verts, out_e, in_e)
        pos = {verts[i]: k for k, i in enumerate(order)}
        for v in verts:
            for u in adj[v]:
                if u in pos and pos[v] > pos[u]:
                    removed.append((u, v))          # (down, up)
    removed.sort()
    rem_set = set((v, u) for (u, v) in removed)     # (up, down)
    # ASAP levels on the cut graph (Kahn)
    indeg = np.zeros(E, dtype=np.int64)
    kept_adj = [[] for _ in range(E)]
    for u, v in zip(up.tolist(), down.tolist()):
        if (u, v) in rem_set:
            continue
        kept_adj[u].append(v)
        indeg[v] += 1
    level = np.zeros(E, dtype=np.int64)
    frontier = [v for v in range(E) if indeg[v] == 0]
    seen = 0
    while frontier:
        nxt = []
        for u in frontier:
            seen += 1
            for v in kept_adj[u]:
                level[v] = max(level[v], level[u] + 1)
                indeg[v] -= 1
                if indeg[v] == 0:
                    nxt.append(v)
        frontier = nxt
    if seen != E:
        raise RuntimeError("cut graph is not acyclic")
    rd = np.array([a for a, _ in removed], dtype=np.int64)
    ru = np.array([b for _, b in removed], dtype=np.int64)
    stats = {
        "edges": int(len(up)),
        "scc_simple": int(sum(1 for s in sizes if s == 2)),
        "scc_large": int(sum(1 for s in sizes if s > 2)),
        "large_sizes": sorted(s for s in sizes if s > 2),
        "removed": int(len(removed)),
        "levels": int(level.max() + 1) if E else 0,
    }
    return GraphResult(up=up, down=down, w=w, z=z, comp=comp, removed_down=rd,
                       removed_up=ru, level=level, stats=stats)
