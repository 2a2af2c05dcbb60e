"""Finite-horizon LQ closed form by the backward Riccati recursion.

Problem: x_k = A x_{k-1} + B u_k (k = 1..H), cost sum_k (x_k - xs)^T Q (x_k - xs)
+ u_k^T R u_k.  The cost-to-go after stage k is x^T P_k x + 2 p_k^T x + const
with P_H = 0, p_H = 0.  Minimising over u_k for a given x_{k-1} = x:

    M = Q + P_k,  m = Q xs - p_k
    u_k = -K_k x + kff_k,   K_k = (R + B^T M B)^{-1} B^T M A,
                            kff_k = (R + B^T M B)^{-1} B^T m
    Abar = A - B K_k,  b = B kff_k
    P_{k-1} = Abar^T M Abar + K_k^T R K_k
    p_{k-1} = Abar^T (M b - m) - K_k^T R kff_k

The first-stage feedback gives u_1* = -K_1 x0 + kff_1, so d u_1*/d x0 = -K_1.
"""
from __future__ import annotations

import numpy as np


def riccati_gains(A, B, Q, R, H, xs):
    nx = A.shape[0]
    P = np.zeros((nx, nx))
    p = np.zeros(nx)
    K = [None] * (H + 1)
    kff = [None] * (H + 1)
    for k in range(H, 0, -1):
        M = Q + P
        m = Q @ xs - p
        S = R + B.T @ M @ B
        K[k] = np.linalg.solve(S, B.T @ M @ A)
        kff[k] = np.linalg.solve(S, B.T @ m)
        Abar = A - B @ K[k]
        b = B @ kff[k]
        P = Abar.T @ M @ Abar + K[k].T @ R @ K[k]
        p = Abar.T @ (M @ b - m) - K[k].T @ R @ kff[k]
    return K, kff


def riccati_solution(A, B, Q, R, H, x0, xs):
    """Optimal (X, U) trajectories, shapes (H, nx) and (H, nu)."""
    K, kff = riccati_gains(A, B, Q, R, H, xs)
    x = np.asarray(x0, float)
    X, U = [], []
    for k in range(1, H + 1):
        u = -K[k] @ x + kff[k]
        x = A @ x + B @ u
        X.append(x)
        U.append(u)
    return np.array(X), np.array(U)
