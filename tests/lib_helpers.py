"""Helpers shared by the library tests: comparisons against the oracle."""
import numpy as np

from oracle.discretization import Discretization
from oracle.graph import direction_graph


def graph_parity(P, wp, directions=None, weighting=None):
    """Return the list of directions whose library graph differs from the
    oracle's (edges, quantised weights, lagged edges, levels)."""
    disc = Discretization(wp)
    wt = wp.weighting if weighting is None else weighting
    bad = []
    for d in (range(disc.D) if directions is None else directions):
        g = direction_graph(disc, d, wt, wp.exact_scc_max)
        up, down, w = P.edges(d)
        o = np.lexsort((g.up, g.down))
        ok = (np.array_equal(up, g.up[o]) and np.array_equal(down, g.down[o])
              and np.array_equal(w, g.w[o]))
        rd, ru = P.removed_edges(d)
        ok = ok and np.array_equal(rd, g.removed_down) and np.array_equal(ru, g.removed_up)
        ok = ok and np.array_equal(P.levels(d), g.level)
        if not ok:
            bad.append(d)
    return bad, disc


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def damping_params(widths, alpha):
    """U-Net parameters whose output is alpha * x0 exactly (linear in the
    residual channel): two channels carry +x0 and -x0 through the full-
    resolution path (leaky ReLU is positively homogeneous, so
    act(act(act(x))) - act(act(act(-x))) = 1.001 x), every coarser layer is
    zero.  With alpha = -0.5 the correction under-relaxes source iteration:
    it lowers the residual, but more slowly than plain sweeps."""
    from oracle import net as N
    parts = []
    for name, i, o, _, _ in N.layer_specs(widths):
        w = np.zeros((o, i, 3, 3, 3))
        if name == "e0a":
            w[0, 0, 1, 1, 1], w[1, 0, 1, 1, 1] = 1.0, -1.0
        elif name in ("e0b", "u0b"):
            w[0, 0, 1, 1, 1], w[1, 1, 1, 1, 1] = 1.0, 1.0
        elif name == "out":
            w[0, 0, 1, 1, 1], w[0, 1, 1, 1, 1] = alpha / 1.001, -alpha / 1.001
        parts += [w.ravel(), np.zeros(o)]
    return np.concatenate(parts)
