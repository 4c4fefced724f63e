"""Training of the learned source-iteration correction (loop control only:
every sweep, network pass, loss, gradient and Adam step runs in the
library's kernels; PyTorch holds the device buffers).

Training pairs come from plain source iteration converged far below the
target tolerance: for a sampled iteration l with phi_{l+1} = S(phi_l), the
input is the scaled element-mean residual mean(phi_{l+1} - phi_l) / s with
the material channels, and the target is mean(phi* - phi_{l+1}) / s (see
``snsw_learn_pair``).
"""
from __future__ import annotations

import time

import numpy as np

from .binding import Net, Problem


def element_grid(P: Problem):
    """(nz, ny, nx) element grid of a problem (nz = 1 in 2D)."""
    nx = list(P.nx) + [1] * (3 - P.dim)
    return nx[2], nx[1], nx[0]


def plain_trajectory(P: Problem, tol: float = 1e-12, max_iters: int = 20000, sample=None, progress=None):
    """Plain source iteration from phi = 0 to `tol`.  Keeps (phi_l, phi_{l+1})
    for the iterations chosen by sample(l) (default: all).  Returns
    (pairs, phi_star, iterations); progress(msg) is called every 500 sweeps."""
    import torch
    En = P.E * P.n
    P.reset()
    cur = torch.zeros(En, dtype=torch.float64, device="cuda")
    nxt = torch.empty_like(cur)
    kept = []
    it = 0
    for it in range(max_iters):
        P.sweep(cur, nxt)
        res = P.residual(nxt, cur)
        if progress is not None and it % 500 == 0:
            progress(f"  sweep {it}: residual {res:.3e}")
        if sample is None or sample(it):
            kept.append((cur.clone(), nxt.clone()))
        cur, nxt = nxt, cur
        if res <= tol:
            break
    return kept, cur.clone(), it + 1


def make_pairs(P: Problem, kept, phi_star):
    """Stacked network inputs X [N][3][E] and targets T [N][E] (float32)."""
    import torch
    N = len(kept)
    X = torch.empty((N, 3, P.E), dtype=torch.float32, device="cuda")
    T = torch.empty((N, P.E), dtype=torch.float32, device="cuda")
    for k, (a, b) in enumerate(kept):
        P.learn_pair(a, b, phi_star, X[k], T[k])
    return X, T


def train(net: Net, grid, X, T, steps: int = 2000, batch: int = 8, lr: float = 1e-3, seed: int = 0,
          lr_final: float = 1e-4, log_every: int = 0):
    """Adam on mean squared error over random minibatches of (X, T).
    The learning rate decays geometrically from lr to lr_final."""
    import torch
    nz, ny, nx = grid
    N = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    xb = torch.empty((batch, 3, nz * ny * nx), dtype=torch.float32, device="cuda")
    tb = torch.empty((batch, nz * ny * nx), dtype=torch.float32, device="cuda")
    yb = torch.empty_like(tb)
    dy = torch.empty_like(tb)
    losses = []
    t0 = time.perf_counter()
    for s in range(steps):
        idx = torch.randint(0, N, (batch,), generator=g).cuda()
        torch.index_select(X, 0, idx, out=xb)
        torch.index_select(T, 0, idx, out=tb)
        net.forward(xb, yb, batch, nz, ny, nx)
        loss = net.loss(yb, tb, dy)
        net.backward(dy)
        rate = lr * (lr_final / lr) ** (s / max(1, steps - 1))
        net.step(lr=rate)
        losses.append(loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            print(f"step {s} loss {loss:.4e} lr {rate:.2e} {time.perf_counter() - t0:.1f}s", flush=True)
    return np.array(losses)
