"""Pins of the mixed-precision model: the float32 factorisation alone is
accurate to about kappa * u32; one FP64 correction brings it to about
(kappa u32)^2, far inside the 1e-5 bar; on local matrices of the curved
mesh the unpivoted factorisation matches LAPACK's solve."""
import numpy as np

import workloads as W
from oracle.discretization import Discretization
from oracle.mixed import lu_nopivot, lu_solve, mixed_solve
from oracle.sweep import build_graphs, sweep


def test_lu_nopivot_float64_matches_lapack():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(20, 9, 9)) + 6 * np.eye(9)
    b = rng.normal(size=(20, 9))
    x = lu_solve(lu_nopivot(A), b)
    assert np.abs(x - np.linalg.solve(A, b[..., None])[..., 0]).max() < 1e-12


def test_refinement_error_scale():
    prob = W.small(dim=2, n=8, r=3, p=3, N=8, amp=0.3 / 8, freq=2, sigma_t=0.5)
    disc = Discretization(prob)
    rng = np.random.default_rng(1)
    for d in (0, 7, 23):
        A = disc.local_matrix(d, np.arange(disc.E))
        b = rng.normal(size=(disc.E, disc.n))
        x = np.linalg.solve(A, b[..., None])[..., 0]
        kappa = np.linalg.cond(A).max()
        u32 = np.finfo(np.float32).eps / 2
        x32 = lu_solve(lu_nopivot(A.astype(np.float32)), b.astype(np.float32)).astype(np.float64)
        xm = mixed_solve(A, b)
        e32 = np.abs(x32 - x).max() / np.abs(x).max()
        em = np.abs(xm - x).max() / np.abs(x).max()
        assert e32 > 1e-9                     # float32 alone is visibly inexact
        assert em < 10 * (kappa * u32) ** 2 + 1e-13
        assert em < e32 / 100


def test_mixed_sweep_within_bar():
    prob = W.small(dim=3, n=3, r=2, p=2, N=4, amp=0.05, c=0.8)
    disc = Discretization(prob)
    gs = build_graphs(disc)
    phi = np.zeros((disc.E, disc.n))
    psi = np.zeros((disc.D, disc.E, disc.n))
    p64, f64 = sweep(disc, gs, phi, psi)
    pm, fm = sweep(disc, gs, phi, psi, solver=mixed_solve)
    err = np.abs(fm - f64).max() / np.abs(f64).max()
    assert err < 1e-9
