"""Jacobi-preconditioned conjugate gradients on a block of right-hand sides,
one independent CG recurrence per column (the step-5 problems are
independent per orbital, Section 3.2). Plain SciPy sparse products; used for
problems too large for a sparse LU and for the CPU-baseline timing.

Stopping rule per column: ||b - A x||_2 <= rtol ||b||_2 (recurrence residual).
"""
from __future__ import annotations

import numpy as np


def jacobi_pcg(A, B, x0=None, rtol=1e-10, maxit=10000, max_iters_total=None):
    B = np.asarray(B, dtype=np.float64)
    one = B.ndim == 1
    if one:
        B = B[:, None]
    n, N = B.shape
    X = np.zeros_like(B) if x0 is None else np.array(x0, dtype=np.float64).reshape(n, N)
    dinv = 1.0 / A.diagonal()
    R = B - A @ X
    Z = dinv[:, None] * R
    Pd = Z.copy()
    rz = np.einsum("ai,ai->i", R, Z)
    bn = np.linalg.norm(B, axis=0)
    bn = np.where(bn == 0, 1.0, bn)
    active = np.linalg.norm(R, axis=0) > rtol * bn
    iters = np.zeros(N, dtype=np.int64)
    for it in range(maxit):
        if not active.any():
            break
        if max_iters_total is not None and it >= max_iters_total:
            break
        Q = A @ Pd
        pq = np.einsum("ai,ai->i", Pd, Q)
        alpha = np.where(active, rz / np.where(pq == 0, 1.0, pq), 0.0)
        X += alpha[None, :] * Pd
        R -= alpha[None, :] * Q
        Z = dinv[:, None] * R
        rz_new = np.einsum("ai,ai->i", R, Z)
        beta = np.where(active, rz_new / np.where(rz == 0, 1.0, rz), 0.0)
        Pd = Z + beta[None, :] * Pd
        rz = rz_new
        iters += active
        active = active & (np.linalg.norm(R, axis=0) > rtol * bn)
    return (X[:, 0] if one else X), iters
