"""The one-state example from the re-solve code listing (Section 3.3).

    dy/dt = 4 sin(u) - y^3,  t in [0, 10] with 15 supports,  y >= 0,  1 <= u <= 3,
    y(0) = y0 (parameter),  minimise the integral of (y - sin(t + tk))^2.

Reading used here: backward difference on the 14 intervals, the integral taken
as dt * sum over stages 1..14 of (y_k - sp_k)^2, y(0) substituted as a parameter.
Decision vector: [y_1, u_1, y_2, u_2, ...].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class ToyOCP:
    def __init__(self, n_supports=15, t_end=10.0):
        self.H = n_supports - 1
        self.dt = t_end / self.H
        self.t = self.dt * np.arange(1, self.H + 1)
        self.ns = 2
        self.n = 2 * self.H
        self.m_c = self.H
        self.m_d = 0
        self.lb = np.tile([0.0, 1.0], self.H)
        self.ub = np.tile([np.inf, 3.0], self.H)
        self.y0 = 1.0
        self.tk = 0.0
        jr, jc = [], []
        for k in range(self.H):
            cols = ([2 * (k - 1)] if k > 0 else []) + [2 * k, 2 * k + 1]
            jr += [k] * len(cols)
            jc += cols
        self.jc_rows, self.jc_cols = np.array(jr), np.array(jc)
        self.jd_rows = self.jd_cols = np.zeros(0, dtype=int)
        self.h_rows = np.repeat(np.arange(self.n), 1)
        self.h_cols = np.arange(self.n)

    def set_parameters(self, y0=None, tk=None, traj=None):
        """traj: the tracked values of stages 1..H given directly (replacing
        sin(t + tk)); None keeps the current choice."""
        if y0 is not None:
            self.y0 = float(y0)
        if tk is not None:
            self.tk = float(tk)
        if traj is not None:
            self.traj = np.array(traj, dtype=np.float64).reshape(self.H)

    traj = None

    def sp(self):
        return np.sin(self.t + self.tk) if self.traj is None else self.traj

    def f(self, y):
        Y = y[0::2]
        return self.dt * np.sum((Y - self.sp()) ** 2)

    def grad(self, y):
        g = np.zeros(self.n, dtype=np.result_type(y, 1.0))
        g[0::2] = 2.0 * self.dt * (y[0::2] - self.sp())
        return g

    def cons_c(self, y):
        Y, U = y[0::2], y[1::2]
        Yp = np.concatenate([[self.y0], Y[:-1]])
        return Y - Yp - self.dt * (4.0 * np.sin(U) - Y ** 3)

    def cons_d(self, y):
        return np.zeros(0, dtype=np.result_type(y, 1.0))

    def jac_c(self, y):
        Y, U = y[0::2], y[1::2]
        data = []
        for k in range(self.H):
            if k > 0:
                data.append(-1.0)
            data.append(1.0 + 3.0 * self.dt * Y[k] ** 2)
            data.append(-4.0 * self.dt * np.cos(U[k]))
        return sp.csr_matrix((np.array(data), (self.jc_rows, self.jc_cols)),
                             shape=(self.m_c, self.n))

    def jac_d(self, y):
        return sp.csr_matrix((self.m_d, self.n))

    def hess(self, y, lam_c, lam_d):
        Y, U = y[0::2], y[1::2]
        diag = np.empty(self.n, dtype=np.result_type(y, lam_c, 1.0))
        diag[0::2] = 2.0 * self.dt + lam_c * 6.0 * self.dt * Y
        diag[1::2] = lam_c * 4.0 * self.dt * np.sin(U)
        return sp.diags(diag).tocsr()

    def initial_guess(self):
        return np.tile([self.y0, 2.0], self.H)

    def parameter_derivatives(self, y):
        """Groups: y0 (1) enters the first state row with coefficient -1; traj
        (H) the tracked value of each stage, in the objective only."""
        Y = y[0::2]
        H, n, dt = self.H, self.n, self.dt
        dc = np.zeros((self.m_c, 1))
        dc[0, 0] = -1.0
        dg = np.zeros((n, H))
        dg[2 * np.arange(H), np.arange(H)] = -2.0 * dt
        dfv = -2.0 * dt * (Y - self.sp())
        return {"y0": (dc, np.zeros((0, 1)), np.zeros((n, 1)), np.zeros(1)),
                "traj": (np.zeros((self.m_c, H)), np.zeros((0, H)), dg, dfv)}

    def u1_index(self):
        return [1]

    def u1(self, y):
        return np.array([y[1]])

    def x1(self, y):
        return np.array([y[0]])
