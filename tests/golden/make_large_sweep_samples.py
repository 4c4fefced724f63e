"""Writes the stored oracle values for the full-size 3D parity tests.

The oracle needs minutes (most of it building the discretisation of 32^3 or
48^3 curved elements) at these sizes, so its results for sampled directions
are stored here instead of being recomputed inside a GPU test.  Everything is
computed by ``oracle/`` from the seeded inputs of ``workloads``; nothing comes
from the library.  Per configuration the file holds:

* ``dirs``: the sampled directions (one per octant, varied position inside
  the octant);
* ``elems``: sampled elements (``workloads.sample_elements``);
* ``psi``: (len(dirs), len(elems), n) angular flux after one lagged sweep
  (eq. laggedSourceIteration) from ``workloads.sweep_inputs`` (seed below),
  restricted to the sampled elements;
* ``graph_sha256``: per sampled direction, the SHA-256 of the oracle's
  edges (up, down, quantised weight; sorted by down, then up), lagged edges
  (down, up) and levels, each as little-endian int64, in that order;
* ``graph_counts``: per sampled direction (edges, lagged edges, levels).

Run from the repository root: ``python tests/golden/make_large_sweep_samples.py``.
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.discretization import Discretization  # noqa: E402
from oracle.graph import direction_graph  # noqa: E402
from oracle.quadrature import level_symmetric  # noqa: E402
from oracle.sweep import lag_masks, sweep  # noqa: E402

SEED = 2024
CONFIGS = {
    # name: (workload, directions, element sample size)
    "c3": (W.c3, [10 * o + k for o, k in enumerate([0, 9, 4, 7, 2, 5, 8, 3])], 384),
    "c5": (W.c5, [21 * o + k for o, k in enumerate([0, 20, 5, 14, 9, 2, 17, 11])], 256),
}


def graph_digest(g) -> tuple:
    o = np.lexsort((g.up, g.down))
    h = hashlib.sha256()
    for a in (g.up[o], g.down[o], g.w[o], g.removed_down, g.removed_up, g.level):
        h.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
    return h.hexdigest(), (len(g.up), len(g.removed_down), int(g.level.max()) + 1)


def make(name: str) -> str:
    make_wp, dirs, count = CONFIGS[name]
    wp = make_wp()
    om, w = level_symmetric(wp.sn_order, wp.dim)
    sel = np.array(dirs)
    disc = Discretization(wp, omega=om[sel], w=w[sel])
    graphs, digests, counts = [], [], []
    for k in range(len(sel)):
        g = direction_graph(disc, k, wp.weighting, wp.exact_scc_max)
        g.mask = lag_masks(disc, g)
        graphs.append(g)
        dg, cn = graph_digest(g)
        digests.append(dg)
        counts.append(cn)
        print(f"{name}: direction {sel[k]}: {cn[0]} edges, {cn[1]} lagged, {cn[2]} levels", flush=True)
    phi0, psi0 = W.sweep_inputs(wp, SEED, sel)
    psi_lag = np.stack([psi0[int(d)] for d in sel])
    psi, _ = sweep(disc, graphs, phi0, psi_lag)
    elems = W.sample_elements(wp, SEED, count)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_sweep_samples.npz")
    np.savez_compressed(out, seed=np.int64(SEED), dirs=sel.astype(np.int64), elems=elems,
                        psi=psi[:, elems, :], graph_sha256=np.array(digests),
                        graph_counts=np.array(counts, dtype=np.int64))
    return out


if __name__ == "__main__":
    for name in (sys.argv[1:] or sorted(CONFIGS)):
        print("wrote", make(name), flush=True)
