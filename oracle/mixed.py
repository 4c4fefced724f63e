"""Mixed-precision local solve (oracle model of the FP32 + FP64 path).

Reading of the mixed mode: the local matrix is rounded to float32 and
factored A32 = L U without pivoting (the symmetric part of A is positive
definite, so the factorisation exists); x0 = (LU)^{-1} b in float32; then one
correction with the FP64 operator, r = b - A x0 in float64 and
x = x0 + (LU)^{-1} r.  The error is about (kappa u32)^2 + kappa u64 for
condition number kappa, against kappa u32 without the correction.
"""
from __future__ import annotations

import numpy as np


def lu_nopivot(A: np.ndarray) -> np.ndarray:
    """Batched LU without pivoting; returns L (unit, below) and U packed."""
    LU = A.copy()
    n = LU.shape[-1]
    for k in range(n - 1):
        l = LU[..., k + 1:, k] / LU[..., k:k + 1, k]
        LU[..., k + 1:, k] = l
        LU[..., k + 1:, k + 1:] -= l[..., :, None] * LU[..., k:k + 1, k + 1:]
    return LU


def lu_solve(LU: np.ndarray, b: np.ndarray) -> np.ndarray:
    n = LU.shape[-1]
    y = b.copy()
    for k in range(n):
        y[..., k] -= np.einsum("...j,...j->...", LU[..., k, :k], y[..., :k])
    x = y
    for k in range(n - 1, -1, -1):
        x[..., k] = (x[..., k] - np.einsum("...j,...j->...", LU[..., k, k + 1:], x[..., k + 1:])) / LU[..., k, k]
    return x


def mixed_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Batched mixed-precision solve of A x = b (A (k,n,n), b (k,n))."""
    LU32 = lu_nopivot(A.astype(np.float32))
    x0 = lu_solve(LU32, b.astype(np.float32)).astype(np.float64)
    r = b - np.einsum("kij,kj->ki", A, x0)
    return x0 + lu_solve(LU32, r.astype(np.float32)).astype(np.float64)
