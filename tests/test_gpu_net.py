"""Learned correction on the GPU (HIP kernels through the C-ABI) against the
CPU FP64 oracle.

The kernels use BF16 weights and FP32 activations and accumulation (the
convolutions are BF16 MFMA tiles: an FP32 activation enters as two BF16
terms hi + lo, which carry it to 2^-16 relative; weight gradients add the
three leading products of the two split operands); the oracle is evaluated
in FP64 with the same BF16-rounded weights (round to nearest even, done here
on the host) and FP32 biases.  The comparison thus measures the split
(about 2^-16 = 1.5e-5 per product) and FP32 accumulation of c*27 <= 864
products (about 864 * 2^-24 = 5e-5 per layer); 12 layers stay within the
1e-3 bar used here (normwise L-infinity).
"""
import numpy as np
import pytest

import workloads as W
from oracle import learned as LR
from oracle import net as N
from oracle.discretization import Discretization
from oracle.sweep import build_graphs
from tests.lib_helpers import rel_err

pytestmark = pytest.mark.gpu
NET_TOL = 1e-3


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_1810_11080_amd import Context
    return Context(device=0)


def bf16_round(a32):
    """float32 -> nearest-even bfloat16 value, as float32."""
    u = np.asarray(a32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def device_weights(theta32, widths):
    """Parameters as the kernels see them: BF16 weights, FP32 biases."""
    out = theta32.astype(np.float64).copy()
    k = 0
    for _, i, o, _, _ in N.layer_specs(widths):
        nw = o * i * 27
        out[k:k + nw] = bf16_round(theta32[k:k + nw]).astype(np.float64)
        k += nw + o
    return out


CASES = [((4, 6, 8), (2, 5, 6, 7)), ((16, 32, 32), (2, 7, 6, 9)), ((4, 6, 8), (3, 1, 9, 8)),
         ((3, 5, 4), (1, 2, 3, 2))]


@pytest.mark.parametrize("widths,shape", CASES, ids=["small-3d", "default-3d", "2d-grid", "tiny-ragged"])
def test_forward_backward_match_oracle(torch, ctx, widths, shape):
    from paper_1810_11080_amd import Net
    B, Z, Y, X = shape
    print(f"net {widths} on {shape}", flush=True)
    net = Net(ctx, widths=widths, seed=1)
    rng = np.random.default_rng(7)
    theta = (N.init_params(widths, seed=3) + 0.02 * rng.standard_normal(N.n_params(widths))).astype(np.float32)
    assert net.n_params == theta.size
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    x = rng.standard_normal((B, 3, Z, Y, X)).astype(np.float32)
    dy = rng.standard_normal((B, 1, Z, Y, X)).astype(np.float32)
    xd = torch.tensor(x.reshape(-1), device="cuda")
    yd = torch.empty(B * Z * Y * X, dtype=torch.float32, device="cuda")
    net.forward(xd, yd, B, Z, Y, X)
    dyd = torch.tensor(dy.reshape(-1), device="cuda")
    dxd = torch.empty_like(xd)
    net.backward(dyd, dxd)
    torch.cuda.synchronize()
    th64 = device_weights(theta, widths)
    y_ref, cache = N.forward(th64, widths, x.astype(np.float64))
    g_ref, dx_ref = N.backward(th64, widths, cache, dy.astype(np.float64), return_dx=True)
    assert rel_err(yd.cpu().numpy().reshape(y_ref.shape), y_ref) <= NET_TOL
    assert rel_err(dxd.cpu().numpy().reshape(x.shape), dx_ref) <= NET_TOL
    g = net.get_grads()
    # layer by layer, so that small early-layer gradients are checked too
    k = 0
    for name, i, o, _, _ in N.layer_specs(widths):
        nw = o * i * 27
        assert rel_err(g[k:k + nw], g_ref[k:k + nw]) <= NET_TOL, name
        assert rel_err(g[k + nw:k + nw + o], g_ref[k + nw:k + nw + o]) <= NET_TOL, name + " bias"
        k += nw + o


def test_loss_and_adam_match_oracle(torch, ctx):
    from paper_1810_11080_amd import Net
    widths = (3, 4, 5)
    net = Net(ctx, widths=widths, seed=2)
    rng = np.random.default_rng(11)
    theta = N.init_params(widths, seed=5).astype(np.float32)
    net.set_params(theta)
    B, Z, Y, X = 2, 4, 5, 3
    x = rng.standard_normal((B, 3, Z, Y, X)).astype(np.float32)
    t = rng.standard_normal((B, 1, Z, Y, X)).astype(np.float32)
    xd = torch.tensor(x.reshape(-1), device="cuda")
    td = torch.tensor(t.reshape(-1), device="cuda")
    yd = torch.empty_like(td)
    dyd = torch.empty_like(td)
    net.forward(xd, yd, B, Z, Y, X)
    loss = net.loss(yd, td, dyd)
    y = yd.cpu().numpy().astype(np.float64)
    ref_loss, ref_dy = N.mse(y, t.reshape(-1).astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-6 * ref_loss
    assert rel_err(dyd.cpu().numpy(), ref_dy) <= 1e-6
    net.backward(dyd)
    g = net.get_grads().astype(np.float64)
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for step in (1, 2, 3):
        net.step(lr=1e-2)
        th, m, v = N.adam_step(th, g, m, v, step, lr=1e-2)
    got = net.get_params().astype(np.float64)
    assert np.abs(got - th).max() <= 1e-6 * max(1.0, np.abs(th).max())


def test_learn_pair_and_correction_match_oracle(torch, ctx):
    """Network input/target from three GPU sweeps against the oracle's
    definitions on the same fluxes."""
    from paper_1810_11080_amd import Problem
    wp = W.c5_reduced(seed=3, nx=4, p=1, sn_order=2)
    P = Problem.from_workload(ctx, wp)
    En = P.E * P.n
    phis = [torch.zeros(En, dtype=torch.float64, device="cuda")]
    for _ in range(3):
        out = torch.empty_like(phis[0])
        P.sweep(phis[-1], out)
        phis.append(out)
    x = torch.empty(3 * P.E, dtype=torch.float32, device="cuda")
    t = torch.empty(P.E, dtype=torch.float32, device="cuda")
    P.learn_pair(phis[1], phis[2], phis[3], x, t)
    torch.cuda.synchronize()
    disc = Discretization(wp)
    h = [p.cpu().numpy().reshape(P.E, P.n) for p in phis]
    xr, tr = LR.training_pair(disc, h[1], h[2], h[3])
    assert rel_err(x.cpu().numpy(), xr.reshape(-1)) <= 1e-6
    assert rel_err(t.cpu().numpy(), tr.reshape(-1)) <= 1e-6


@pytest.mark.parametrize("every", [1, 3])
def test_preconditioned_solve_matches_oracle(torch, ctx, every):
    """Source iteration with a (random) network on the GPU and in the oracle
    converge to the same fixed point; the safeguard keeps it convergent."""
    from paper_1810_11080_amd import Net, Problem
    wp = W.c5_reduced(seed=4, nx=4, p=1, sn_order=2)
    widths = (3, 4, 5)
    theta = N.init_params(widths, seed=6).astype(np.float32)
    net = Net(ctx, widths=widths)
    net.set_params(theta)
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    rep = P.solve(phi, tol=1e-11, max_iters=20000, precond=net, precond_every=every)
    disc = Discretization(wp)
    gs = build_graphs(disc)
    phi_ref, hist, ncorr = LR.preconditioned_si(disc, gs, device_weights(theta, widths), widths, 1e-11, 20000,
                                                every=every)
    assert rep["residual"] <= 1e-11 and hist[-1] <= 1e-11
    assert rep["n_corrected"] > 0 and ncorr > 0
    assert rel_err(phi.cpu().numpy().reshape(P.E, P.n), phi_ref) <= 1e-8


def test_trained_network_gains(torch, ctx):
    """Train on plain-SI pairs of three seeds of the two-material c = 0.99
    family (12^3 Q2, p = 1, S4), then solve a held-out seed to 1e-8 with and
    without the network: fewer sweeps and less wall time with it."""
    import time
    from paper_1810_11080_amd import Net, Problem
    from paper_1810_11080_amd import learn as L
    Xs, Ts = [], []
    for seed in range(3):
        P = Problem.from_workload(ctx, W.c5_reduced(seed=seed, nx=12, p=1, sn_order=4))
        kept, star, its = L.plain_trajectory(P, tol=1e-12, max_iters=20000, sample=lambda l: l % 3 == 0)
        X, T = L.make_pairs(P, kept, star)
        Xs.append(X)
        Ts.append(T)
        print(f"training seed {seed}: {its} plain sweeps, {len(kept)} pairs", flush=True)
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    net = Net(ctx, widths=(16, 32, 32), seed=0)
    losses = L.train(net, (12, 12, 12), X, T, steps=2500, batch=8, lr=2e-3, lr_final=1e-4)
    assert losses[-100:].mean() < 0.2 * losses[:10].mean()
    P = Problem.from_workload(ctx, W.c5_reduced(seed=100, nx=12, p=1, sn_order=4))
    out = {}
    for name, pre in (("plain", None), ("learned", net)):
        best = None
        for _ in range(2):
            P.reset()
            phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
            t0 = time.perf_counter()
            rep = P.solve(phi, tol=1e-8, max_iters=20000, precond=pre, precond_every=40)
            dt = time.perf_counter() - t0
            best = (rep["iterations"], dt) if best is None or dt < best[1] else best
        out[name] = best
    print(out, flush=True)
    assert out["learned"][0] < 0.8 * out["plain"][0]
    assert out["learned"][1] < out["plain"][1]


def test_safeguard_rejects_slower_correction(torch, ctx):
    """The library's safeguard at period 1 (the solve's default): an
    under-relaxing network is rejected three times and switched off, as in
    the oracle, and the solve keeps the plain iteration count within 3."""
    from paper_1810_11080_amd import Net, Problem
    from tests.lib_helpers import damping_params
    widths = (2, 2, 2)
    wp = W.make_problem("damp", 2, (6, 6), 2, 1, 4, 0.05, 1, 1.0, 0.9, 1.0)
    theta = damping_params(widths, -0.5).astype(np.float32)
    net = Net(ctx, widths=widths)
    net.set_params(theta)
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    plain = P.solve(phi, tol=1e-10, max_iters=2000)
    P.reset()
    phi_c = torch.zeros_like(phi)
    rep = P.solve(phi_c, tol=1e-10, max_iters=2000, precond=net, precond_every=1)
    disc = Discretization(wp)
    gs = build_graphs(disc)
    _, hist, ncorr = LR.preconditioned_si(disc, gs, device_weights(theta, widths), widths, 1e-10, 2000, every=1)
    print(f"plain {plain['iterations']}, corrected {rep['iterations']} ({rep['n_corrected']} applied, "
          f"{rep['n_rejected']} rejected), oracle {len(hist)}", flush=True)
    assert rep["n_rejected"] == LR.MAX_REJECTIONS and rep["n_corrected"] == ncorr == LR.MAX_REJECTIONS
    assert rep["iterations"] == len(hist)
    assert rep["iterations"] <= plain["iterations"] + 3
    assert rel_err(phi_c.cpu().numpy(), phi.cpu().numpy()) <= 1e-9


def test_default_network_correction_matches_oracle(torch, ctx):
    """The default 16/32/32 network applied inside the solve on a 12^3
    element grid (two plain sweeps, then the correction): the correction
    phi_corrected - phi~ matches the oracle's (FP64 with the same BF16
    weights) to the network bar, and phi~ itself to FP64 rounding."""
    from paper_1810_11080_amd import Net, Problem
    from oracle.sweep import sweep
    widths = (16, 32, 32)
    wp = W.c5_reduced(seed=7, nx=12, p=1, sn_order=2)
    theta = (N.init_params(widths, seed=9)).astype(np.float32)
    net = Net(ctx, widths=widths)
    net.set_params(theta)
    P = Problem.from_workload(ctx, wp)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    rep = P.solve(phi, tol=0.0, max_iters=2, precond=net, precond_every=2, raise_on_not_converged=False)
    assert rep["n_corrected"] == 1
    disc = Discretization(wp)
    gs = build_graphs(disc)
    o_phi = np.zeros((disc.E, disc.n))
    o_psi = np.zeros((disc.D, disc.E, disc.n))
    for _ in range(2):
        o_prev = o_phi
        o_psi, o_phi = sweep(disc, gs, o_phi, o_psi)
    ref = LR.correction(disc, device_weights(theta, widths), widths, o_prev, o_phi)
    got = phi.cpu().numpy().reshape(P.E, P.n)
    assert np.abs(ref - o_phi).max() > 1e-3 * np.abs(o_phi).max()    # a correction of some size
    assert rel_err(got - o_phi, ref - o_phi) <= NET_TOL
