"""Linear-quadratic test family (oracle side).

    x_k = A x_{k-1} + B u_k,  k = 1..H,  x_0 = x0 (parameter)
    minimise  sum_k (x_k - xs)^T Q (x_k - xs) + u_k^T R u_k
    optional box bounds on x and u (default: none)

Transcribed like the NMPC families: c_k = x_k - A x_{k-1} - B u_k = 0, decision
vector stage-major [x_1, u_1, x_2, u_2, ...].  With no active bounds the
solution has the finite-horizon Riccati closed form (see ``riccati``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from workloads.generators import random_lq  # noqa: F401  (seeded inputs, shared)


class LQOCP:
    def __init__(self, A, B, Q, R, H, xs=None, x_bounds=None, u_bounds=None):
        self.A, self.B = np.asarray(A, float), np.asarray(B, float)
        self.Q, self.R = np.asarray(Q, float), np.asarray(R, float)
        self.nx, self.nu = self.B.shape
        self.H = int(H)
        self.ns = self.nx + self.nu
        self.n = self.H * self.ns
        self.m_c = self.H * self.nx
        self.m_d = 0
        self.xs = np.zeros(self.nx) if xs is None else np.asarray(xs, float)
        self.x0 = np.zeros(self.nx)
        lo = np.full(self.ns, -np.inf)
        hi = np.full(self.ns, np.inf)
        if x_bounds is not None:
            lo[:self.nx], hi[:self.nx] = x_bounds
        if u_bounds is not None:
            lo[self.nx:], hi[self.nx:] = u_bounds
        self.lb, self.ub = np.tile(lo, self.H), np.tile(hi, self.H)
        # Jacobian: full dense blocks I, -B, -A (structural)
        jr, jc = [], []
        for k in range(self.H):
            for i in range(self.nx):
                cols = []
                if k > 0:
                    cols += [(k - 1) * self.ns + j for j in range(self.nx)]
                cols += [k * self.ns + j for j in range(self.ns)]
                jr += [k * self.nx + i] * len(cols)
                jc += cols
        self.jc_rows, self.jc_cols = np.array(jr), np.array(jc)
        self.jd_rows = self.jd_cols = np.zeros(0, dtype=int)
        hr, hc = [], []
        for k in range(self.H):
            o = k * self.ns
            for i in range(self.ns):
                for j in range(i + 1):
                    hr.append(o + i)
                    hc.append(o + j)
        self.h_rows, self.h_cols = np.array(hr), np.array(hc)

    def set_parameters(self, x0=None, xs=None):
        if x0 is not None:
            self.x0 = np.asarray(x0, float).copy()
        if xs is not None:
            self.xs = np.asarray(xs, float).copy()

    def split(self, y):
        Y = y.reshape(self.H, self.ns)
        return Y[:, :self.nx], Y[:, self.nx:]

    def f(self, y):
        X, U = self.split(y)
        E = X - self.xs
        return np.sum((E @ self.Q) * E) + np.sum((U @ self.R) * U)

    def grad(self, y):
        X, U = self.split(y)
        G = np.concatenate([2.0 * (X - self.xs) @ self.Q, 2.0 * U @ self.R], axis=1)
        return G.reshape(-1)

    def cons_c(self, y):
        X, U = self.split(y)
        Xp = np.vstack([self.x0[None, :], X[:-1]])
        return (X - Xp @ self.A.T - U @ self.B.T).reshape(-1)

    def cons_d(self, y):
        return np.zeros(0, dtype=np.result_type(y, 1.0))

    def jac_c(self, y):
        vals = {}
        for k in range(self.H):
            for i in range(self.nx):
                r = k * self.nx + i
                if k > 0:
                    for j in range(self.nx):
                        vals[(r, (k - 1) * self.ns + j)] = -self.A[i, j]
                for j in range(self.nx):
                    vals[(r, k * self.ns + j)] = 1.0 if i == j else 0.0
                for j in range(self.nu):
                    vals[(r, k * self.ns + self.nx + j)] = -self.B[i, j]
        data = np.array([vals[(r, c)] for r, c in zip(self.jc_rows, self.jc_cols)])
        return sp.csr_matrix((data, (self.jc_rows, self.jc_cols)), shape=(self.m_c, self.n))

    def jac_d(self, y):
        return sp.csr_matrix((self.m_d, self.n))

    def hess(self, y, lam_c, lam_d):
        blk = np.zeros((self.ns, self.ns))
        blk[:self.nx, :self.nx] = 2.0 * self.Q
        blk[self.nx:, self.nx:] = 2.0 * self.R
        return sp.block_diag([blk] * self.H).tocsr()

    def parameter_derivatives(self, y):
        """Groups: x0 (nx) enters c_1 = x_1 - A x0 - B u_1; xs (nx) enters f."""
        X, U = self.split(y)
        nx, n = self.nx, self.n
        dc = np.zeros((self.m_c, nx))
        dc[:nx, :] = -self.A
        dg = np.zeros((n, nx))
        for k in range(self.H):
            dg[k * self.ns:k * self.ns + nx, :] = -2.0 * self.Q
        dfv = -2.0 * np.sum((X - self.xs) @ self.Q, axis=0)
        return {"x0": (dc, np.zeros((0, nx)), np.zeros((n, nx)), np.zeros(nx)),
                "xs": (np.zeros((self.m_c, nx)), np.zeros((0, nx)), dg, dfv)}

    def u1_index(self):
        return list(range(self.nx, self.ns))

    def initial_guess(self):
        y = np.zeros(self.n)
        for k in range(self.H):
            y[k * self.ns:k * self.ns + self.nx] = self.x0
        return y

    def u1(self, y):
        return np.array(y[self.nx:self.ns])

    def x1(self, y):
        return np.array(y[:self.nx])
