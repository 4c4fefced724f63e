"""Batched sweeps (many independent problems, merged per-class schedules,
autotuned schedule choice, hipGraph replay) through the C-ABI.

Bars: each problem of a batch matches the CPU FP64 oracle within 1e-10
(FP64) or 1e-5 (mixed precision) relative L-infinity error after every
sweep; a batch sweep reproduces the single-problem sweep of the same kernel
bit for bit (the same pairs run the same arithmetic); graph replays equal
eager launches bit for bit.  The 64-problem batch drawn from seed 0 is
checked at full size in the launch configuration the benchmark times.
"""
import numpy as np
import pytest

import workloads as W
from oracle.discretization import Discretization
from oracle.sweep import build_graphs, sweep as oracle_sweep
from tests.lib_helpers import rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-10
MIXED_TOL = 1e-5
AUTO, PERSISTENT, LEVELS = 0, 1, 2


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.fixture(scope="module")
def ctx(torch):
    from paper_1810_11080_amd import Context
    return Context(device=0)


def seeded_phi(wp, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(wp.n_elements, (wp.p + 1) ** wp.dim))


def oracle_run(wp, phi0, K):
    disc = Discretization(wp)
    gs = build_graphs(disc)
    phi = phi0.copy()
    psi = np.zeros((disc.D, disc.E, disc.n))
    out = []
    for _ in range(K):
        psi, phi = oracle_sweep(disc, gs, phi, psi)
        out.append(phi)
    return out


def batch_run(torch, B, problems, phi0s, K):
    """K batch sweeps from phi0s; returns [sweep][problem] host arrays."""
    ins = [torch.tensor(p0.reshape(-1), dtype=torch.float64, device="cuda") for p0 in phi0s]
    outs = [torch.empty_like(t) for t in ins]
    res = []
    for _ in range(K):
        B.sweep(ins, outs)
        B.synchronize()
        res.append([o.cpu().numpy().reshape(P.E, P.n).copy() for o, P in zip(outs, problems)])
        ins, outs = outs, ins
    return res


def single_run(torch, P, phi0, K):
    phi = torch.tensor(phi0.reshape(-1), dtype=torch.float64, device="cuda")
    out = torch.empty_like(phi)
    res = []
    for _ in range(K):
        P.sweep(phi, out)
        P.synchronize()
        res.append(out.cpu().numpy().reshape(P.E, P.n).copy())
        phi, out = out, phi
    return res


# ragged mix: 2D p = 1, 2, 3 (two of them in one class), 3D p = 1, 2,
# mixed-precision members (2D p = 3 and p = 2: persistent kernels with FP32
# inverses when the batch sweeps persistently), cyclic graphs, an isotropic
# inflow boundary
MIX = [
    ("cyc2d_p1", lambda: W.small(dim=2, n=12, r=3, p=1, N=8, amp=0.3 / 12, freq=3, c=0.7), 0),
    ("cyc2d_p3", lambda: W.make_problem("cyc_p3", 2, (17, 11), 3, 3, 8, 0.3 / 17, 4,
                                        np.linspace(0.5, 4, 187), 0.6, 1.0), 0),
    ("c1", W.c1, 0),
    ("inflow2d_p2", lambda: W.small(dim=2, n=(9, 6), r=2, p=2, N=6, amp=0.04, c=0.3,
                                    bc_kind=W.ISO_CONST, psi_inc=0.6), 0),
    ("p3_small", lambda: W.small(dim=2, n=5, r=2, p=3, N=4, amp=0.05, c=0.9, sigma_t=3.0), 0),
    ("warp3d_p1", lambda: W.small(dim=3, n=(4, 3, 5), r=2, p=1, N=4, amp=0.08, freq=1), 0),
    ("warp3d_p2", lambda: W.make_problem("w3p2", 3, (4, 4, 3), 2, 2, 4, 0.07, 1,
                                         np.linspace(0.5, 5, 48), 0.8, 1.0), 0),
    ("mixed2d_p3", lambda: W.small(dim=2, n=6, r=2, p=3, N=6, amp=0.05, c=0.8), 1),
    ("mixed2d_p2", lambda: W.small(dim=2, n=(7, 9), r=3, p=2, N=8, amp=0.3 / 9, freq=2, c=0.9), 1),
]


@pytest.fixture(scope="module")
def mix_reference():
    wps = [f() for _, f, _ in MIX]
    phi0s = [seeded_phi(wp, 10 + k) for k, wp in enumerate(wps)]
    ref = [oracle_run(wp, p0, 3) for wp, p0 in zip(wps, phi0s)]
    return wps, phi0s, ref


@pytest.mark.parametrize("schedule,use_graph", [(AUTO, True), (PERSISTENT, True), (LEVELS, True),
                                                (PERSISTENT, False)],
                         ids=["auto-graph", "persistent-graph", "levels-graph", "persistent-eager"])
def test_batch_matches_oracle(torch, ctx, mix_reference, schedule, use_graph):
    from paper_1810_11080_amd import Batch, Problem
    wps, phi0s, ref = mix_reference
    print(f"batch of {len(wps)} problems, schedule {schedule}, graph {use_graph}", flush=True)
    problems = [Problem.from_workload(ctx, wp, precision=prec, schedule=LEVELS if prec else AUTO)
                for wp, (_, _, prec) in zip(wps, MIX)]
    B = Batch(ctx, problems, schedule=schedule, use_graph=use_graph, tune_reps=1)
    classes = B.classes()
    assert sum(c["n_problems"] for c in classes) == len(problems)
    assert len(classes) == 7
    if schedule == PERSISTENT:   # lattices only: every class, mixed ones included, sweeps persistently
        assert all(c["persistent"] == 1 for c in classes)
        assert sum(c["precision"] == 1 for c in classes) == 2
    got = batch_run(torch, B, problems, phi0s, 3)
    for k, (name, _, prec) in enumerate(MIX):
        tol = MIXED_TOL if prec else TOL
        for it in range(3):
            err = rel_err(got[it][k], ref[k][it])
            assert err <= tol, (name, it, err)
    B.close()


def test_batch_interleaved_with_single_sweeps(torch, ctx, mix_reference):
    """A member swept on its own between batch sweeps keeps one consistent
    lagged state: batch, single, batch == three oracle sweeps."""
    from paper_1810_11080_amd import Batch, Problem
    wps, phi0s, ref = mix_reference
    sel = [0, 1, 5]
    problems = [Problem.from_workload(ctx, wps[k]) for k in sel]
    B = Batch(ctx, problems, schedule=AUTO, use_graph=True, tune_reps=1)
    ins = [torch.tensor(phi0s[k].reshape(-1), dtype=torch.float64, device="cuda") for k in sel]
    mids = [torch.empty_like(t) for t in ins]
    B.sweep(ins, mids)
    outs = [torch.empty_like(t) for t in ins]
    for P, a, b in zip(problems, mids, outs):
        P.sweep(a, b)
    fin = [torch.empty_like(t) for t in ins]
    B.sweep(outs, fin)
    B.synchronize()
    for j, k in enumerate(sel):
        assert rel_err(mids[j].cpu().numpy().reshape(ref[k][0].shape), ref[k][0]) <= TOL
        assert rel_err(outs[j].cpu().numpy().reshape(ref[k][1].shape), ref[k][1]) <= TOL
        assert rel_err(fin[j].cpu().numpy().reshape(ref[k][2].shape), ref[k][2]) <= TOL
    B.close()


def test_batch_rejects_bad_input(torch, ctx):
    from paper_1810_11080_amd import Batch, Problem, SnswError
    wp = W.c1()
    P = Problem.from_workload(ctx, wp)
    with pytest.raises(SnswError) as ei:
        Batch(ctx, [P, P])
    assert ei.value.code == -1
    B = Batch(ctx, [P], schedule=LEVELS)
    phi = torch.zeros(P.E * P.n, dtype=torch.float64, device="cuda")
    with pytest.raises(SnswError):
        B.sweep([phi], [phi])          # aliasing input and output
    with pytest.raises(ValueError):
        B.sweep([phi, phi], [phi])
    B.close()


def c4_small(seed=7, count=12):
    """Problems drawn like the 64-problem batch, with 16..32 elements a side."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        m = int(rng.integers(16, 33))
        p = int(rng.integers(1, 4))
        N = 2 * int(rng.integers(2, 7))
        st = float(10.0 ** rng.uniform(-1.0, 1.0))
        c = float(rng.uniform(0.0, 0.95))
        out.append(W.make_problem(f"c4s_{b}", 2, (m, m), 2, p, N, 0.05, 1, st, c, 1.0, tol=1e-8))
    return out


@pytest.mark.parametrize("schedule", [PERSISTENT, LEVELS], ids=["persistent", "levels"])
def test_batch_bit_exact_vs_single(torch, ctx, schedule):
    from paper_1810_11080_amd import Batch, Problem
    wps = c4_small()
    phi0s = [seeded_phi(wp, 100 + k) for k, wp in enumerate(wps)]
    print(f"c4-like batch of {len(wps)}, schedule {schedule}", flush=True)
    single = []
    for wp, p0 in zip(wps, phi0s):
        P = Problem.from_workload(ctx, wp, schedule=schedule)
        single.append(single_run(torch, P, p0, 2))
        P.close()
    problems = [Problem.from_workload(ctx, wp) for wp in wps]
    for use_graph in (True, False):
        for P in problems:
            P.reset()
        B = Batch(ctx, problems, schedule=schedule, use_graph=use_graph)
        got = batch_run(torch, B, problems, phi0s, 2)
        for k in range(len(wps)):
            for it in range(2):
                assert np.array_equal(got[it][k], single[k][it]), (k, it, use_graph)
        B.close()


def test_c4_full_batch(torch, ctx):
    """The 64-problem batch (seed 0) as the benchmark runs it: autotuned,
    graph replay.  Every member is compared bit for bit with its own
    single-problem sweep under the schedule the tuner picked for its class;
    the two smallest members are also compared with the oracle."""
    from paper_1810_11080_amd import Batch, Problem
    wps = W.c4()
    print(f"full batch: {len(wps)} problems", flush=True)
    phi0s = [seeded_phi(wp, 1000 + k) for k, wp in enumerate(wps)]
    problems = [Problem.from_workload(ctx, wp) for wp in wps]
    B = Batch(ctx, problems, schedule=AUTO, use_graph=True)
    classes = B.classes()
    print(classes, flush=True)
    got = batch_run(torch, B, problems, phi0s, 2)
    B.close()
    sched_of = {}
    for c in classes:
        sched_of[(c["dim"], c["dg_order"])] = PERSISTENT if c["persistent"] else LEVELS
    work = [wp.n_elements * (wp.p + 1) ** 2 * wp.n_dirs for wp in wps]
    smallest = list(np.argsort(work)[:2])
    sample = sorted(set(smallest) | set(range(0, 64, 9)))
    for k in sample:
        wp = wps[k]
        S = Problem.from_workload(ctx, wp, schedule=sched_of[(2, wp.p)])
        one = single_run(torch, S, phi0s[k], 2)
        S.close()
        for it in range(2):
            assert np.array_equal(got[it][k], one[it]), (k, it)
    for k in smallest:
        ref = oracle_run(wps[k], phi0s[k], 2)
        for it in range(2):
            assert rel_err(got[it][k], ref[it]) <= TOL, (k, it)
