"""The allocation-free training-pair entry point (static device scratch)
against snsw_learn_pair on the same fluxes: two calls in a row, the second
on a smaller problem, so stale scratch contents of the first call would
show.  Both run the same kernels on the same inputs, so the results must be
identical bit for bit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


def fluxes(torch, P, sweeps=3):
    En = P.E * P.n
    phis = [torch.zeros(En, dtype=torch.float64, device="cuda")]
    for _ in range(sweeps):
        out = torch.empty_like(phis[0])
        P.sweep(phis[-1], out)
        phis.append(out)
    torch.cuda.synchronize()
    return phis


def pair(torch, P, phis, noalloc, target=True):
    x = torch.full((3 * P.E,), float("nan"), dtype=torch.float32, device="cuda")
    t = torch.full((P.E,), float("nan"), dtype=torch.float32, device="cuda") if target else None
    f = P.learn_pair_noalloc if noalloc else P.learn_pair
    f(phis[1], phis[2], phis[3] if target else None, x, t)
    torch.cuda.synchronize()
    return x.cpu().numpy(), (t.cpu().numpy() if target else None)


def test_noalloc_learn_pair_matches_allocating_one(torch):
    from paper_1810_11080_amd import Context, Problem
    ctx = Context(device=0)
    big = Problem.from_workload(ctx, W.c5_reduced(seed=7, nx=10, p=2, sn_order=4))
    small = Problem.from_workload(ctx, W.c5_reduced(seed=8, nx=5, p=1, sn_order=2))
    assert small.E < big.E
    cases = [(big, True), (small, True), (small, False)]
    for P, target in cases:
        print(f"learn_pair_noalloc: E={P.E} n={P.n} target={target}", flush=True)
        phis = fluxes(torch, P)
        xr, tr = pair(torch, P, phis, noalloc=False, target=target)
        x, t = pair(torch, P, phis, noalloc=True, target=target)
        assert np.all(np.isfinite(x)) and np.array_equal(x, xr), P.E
        if target:
            assert np.all(np.isfinite(t)) and np.array_equal(t, tr), P.E
        assert np.abs(x[:P.E]).max() == 1.0   # scaled by its own maximum
    small.close()
    big.close()
