"""Transcribed distillation-column OCP (oracle side).

Follows the distillation case study of Section 4.1 in structure: tray liquid
mole fractions with constant molar overflow and constant relative volatility,
a total condenser and a reboiler, feed on one tray, controlled by reflux R and
boilup V, discretized by backward (implicit) Euler as in the paper's setup.

States per stage: x_0 (condenser / distillate), x_1..x_N (trays, top to
bottom), x_{N+1} (reboiler / bottoms).  Controls per stage: (R, V).
Flows: D = V - R, B = R + F - V; VLE y(x) = a x / (1 + (a - 1) x).

    dx_0/dt     = V (y_1 - x_0)
    dx_i/dt     = Lin_i x_{i-1} - Lout_i x_i + V (y_{i+1} - y_i) + [i = f] F zF
                  Lin_i = R (i <= f) else R + F;  Lout_i = R (i < f) else R + F
    dx_{N+1}/dt = (R + F) x_N - V y_{N+1} - B x_{N+1}

Transcription (stages k = 1..H, x at stage 0 is the measured parameter x0):
    c_k = x_k - x_{k-1} - dt * rhs(x_k, u_k; zF_k) = 0
Objective: sum_k (x_{k,0} - xD*)^2 + (x_{k,N+1} - xB*)^2 + rho |u_k - u_{k-1}|^2
with u_0 the previously applied control (a parameter).
Inequalities (g <= 0 form): R - V <= 0 (D >= 0), V - R - F <= 0 (B >= 0).
Bounds: x in [0, 1], R, V in [0.5, 5].
Control horizon (Section 3.1, eqs. 4-5): with Hc < H the controls are held at
their value of stage Hc after it.  The hold is written as u_k - u_{k-1} = 0 for
stages k = Hc+1..H (1-based), the same feasible set as u_k = u_Hc; these
equality rows follow the H*nx dynamics rows, controls R then V per stage.

Decision vector y is stage-major: stage k occupies y[k*ns:(k+1)*ns] with
ns = N + 4, laid out [x_0 .. x_{N+1}, R, V].

All functions accept complex y so derivatives can be checked by complex step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class DistillationOCP:
    def __init__(self, N, H, dt, alpha, F=1.0, xD_sp=0.95, xB_sp=0.05, rho=1e-2,
                 x_lo=0.0, x_hi=1.0, u_lo=0.5, u_hi=5.0, Hc=None):
        self.N, self.H, self.dt = int(N), int(H), float(dt)
        self.Hc = self.H if Hc is None or Hc <= 0 or Hc >= H else int(Hc)   # control horizon (stages)
        self.alpha, self.F, self.rho = float(alpha), float(F), float(rho)
        self.nx = self.N + 2
        self.nu = 2
        self.ns = self.nx + self.nu
        self.n = self.H * self.ns
        self.m_dyn = self.H * self.nx
        self.m_c = self.m_dyn + self.nu * (self.H - self.Hc)
        self.m_d = 2 * self.H
        self.fd = self.N // 2
        lb = np.empty(self.n)
        ub = np.empty(self.n)
        for k in range(self.H):
            o = k * self.ns
            lb[o:o + self.nx], ub[o:o + self.nx] = x_lo, x_hi
            lb[o + self.nx:o + self.ns], ub[o + self.nx:o + self.ns] = u_lo, u_hi
        self.lb, self.ub = lb, ub
        # parameters
        self.x0 = np.full(self.nx, 0.5)
        self.zF = np.full(self.H, 0.5)
        self.u_prev = np.array([2.0, 2.5])
        self.xD_sp, self.xB_sp = float(xD_sp), float(xB_sp)
        self._build_patterns()

    @classmethod
    def from_workload(cls, w):
        m = cls(w.N, w.H, w.dt, w.alpha, F=w.F, xD_sp=w.xD_sp, xB_sp=w.xB_sp,
                rho=w.rho, x_lo=w.x_lo, x_hi=w.x_hi, u_lo=w.u_lo, u_hi=w.u_hi, Hc=getattr(w, "Hc", None))
        return m

    def set_parameters(self, x0=None, zF=None, u_prev=None, setpoint=None):
        if x0 is not None:
            self.x0 = np.array(x0, dtype=np.float64).reshape(self.nx)
        if zF is not None:
            self.zF = np.array(zF, dtype=np.float64).reshape(self.H)
        if u_prev is not None:
            self.u_prev = np.array(u_prev, dtype=np.float64).reshape(2)
        if setpoint is not None:
            self.xD_sp, self.xB_sp = float(setpoint[0]), float(setpoint[1])

    # ---- index helpers -------------------------------------------------
    def ix(self, k, i):
        """Index of x_i at stage k (0-based stage)."""
        return k * self.ns + i

    def iR(self, k):
        return k * self.ns + self.nx

    def iV(self, k):
        return k * self.ns + self.nx + 1

    def split(self, y):
        Y = y.reshape(self.H, self.ns)
        return Y[:, :self.nx], Y[:, self.nx], Y[:, self.nx + 1]

    def _vle(self, x):
        a = self.alpha
        g = 1.0 + (a - 1.0) * x
        return a * x / g, a / g ** 2, -2.0 * a * (a - 1.0) / g ** 3

    # ---- model right-hand side ----------------------------------------
    def rhs(self, X, R, V, zF):
        """dx/dt for every stage: X (H, nx), R, V, zF (H,) -> (H, nx)."""
        N, F, fd = self.N, self.F, self.fd
        yv, _, _ = self._vle(X)
        out = np.zeros_like(X + 0.0 * R[:, None])
        out[:, 0] = V * (yv[:, 1] - X[:, 0])
        for i in range(1, N + 1):
            lin = R if i <= fd else R + F
            lout = R if i < fd else R + F
            out[:, i] = lin * X[:, i - 1] - lout * X[:, i] + V * (yv[:, i + 1] - yv[:, i])
            if i == fd:
                out[:, i] = out[:, i] + F * zF
        out[:, N + 1] = (R + F) * X[:, N] - V * yv[:, N + 1] - (R + F - V) * X[:, N + 1]
        return out

    # ---- NLP functions -------------------------------------------------
    def f(self, y):
        X, R, V = self.split(y)
        Rp = np.concatenate([[self.u_prev[0]], R[:-1]])
        Vp = np.concatenate([[self.u_prev[1]], V[:-1]])
        return (np.sum((X[:, 0] - self.xD_sp) ** 2) + np.sum((X[:, -1] - self.xB_sp) ** 2)
                + self.rho * (np.sum((R - Rp) ** 2) + np.sum((V - Vp) ** 2)))

    def grad(self, y):
        X, R, V = self.split(y)
        G = np.zeros((self.H, self.ns), dtype=np.result_type(y, 1.0))
        G[:, 0] = 2.0 * (X[:, 0] - self.xD_sp)
        G[:, self.nx - 1] = 2.0 * (X[:, -1] - self.xB_sp)
        for col, U, up in ((self.nx, R, self.u_prev[0]), (self.nx + 1, V, self.u_prev[1])):
            Up = np.concatenate([[up], U[:-1]])
            d = 2.0 * self.rho * (U - Up)
            G[:, col] += d
            G[:-1, col] -= d[1:]
        return G.reshape(-1)

    def cons_c(self, y):
        X, R, V = self.split(y)
        Xp = np.vstack([self.x0[None, :], X[:-1]])
        dyn = (X - Xp - self.dt * self.rhs(X, R, V, self.zF)).reshape(-1)
        hc = self.Hc
        hold = np.stack([R[hc:] - R[hc - 1:-1], V[hc:] - V[hc - 1:-1]], axis=1).reshape(-1)
        return np.concatenate([dyn, hold])

    def cons_d(self, y):
        _, R, V = self.split(y)
        d = np.empty((self.H, 2), dtype=np.result_type(y, 1.0))
        d[:, 0] = R - V
        d[:, 1] = V - R - self.F
        return d.reshape(-1)

    # ---- structural patterns and derivative values --------------------
    def _build_patterns(self):
        """Structural Jacobian / Hessian entry lists (values filled per call)."""
        N, nx, H = self.N, self.nx, self.H
        jr, jc = [], []
        for k in range(H):
            for i in range(nx):
                row = k * nx + i
                cols = set()
                if k > 0:
                    cols.add(self.ix(k - 1, i))
                for ii in range(max(0, i - 1), min(nx, i + 2)):
                    cols.add(self.ix(k, ii))
                if i > 0:
                    cols.add(self.iR(k))
                cols.add(self.iV(k))
                for c in sorted(cols):
                    jr.append(row)
                    jc.append(c)
        for k in range(self.Hc, H):       # holds: u_k - u_{k-1}
            for j, idx in enumerate((self.iR, self.iV)):
                row = self.m_dyn + 2 * (k - self.Hc) + j
                jr += [row, row]
                jc += [idx(k - 1), idx(k)]
        self.jc_rows, self.jc_cols = np.array(jr), np.array(jc)
        dr, dc = [], []
        for k in range(H):
            for r in range(2):
                dr += [2 * k + r, 2 * k + r]
                dc += [self.iR(k), self.iV(k)]
        self.jd_rows, self.jd_cols = np.array(dr), np.array(dc)
        # Hessian of the Lagrangian, lower triangle (row >= col)
        hr, hc = [], []
        for k in range(H):
            for i in range(nx):
                hr.append(self.ix(k, i)); hc.append(self.ix(k, i))
            for i in range(nx):
                hr.append(self.iR(k)); hc.append(self.ix(k, i))
            hr.append(self.iR(k)); hc.append(self.iR(k))
            for i in range(nx):
                hr.append(self.iV(k)); hc.append(self.ix(k, i))
            hr.append(self.iV(k)); hc.append(self.iV(k))
            if k > 0:
                hr.append(self.iR(k)); hc.append(self.iR(k - 1))
                hr.append(self.iV(k)); hc.append(self.iV(k - 1))
        self.h_rows, self.h_cols = np.array(hr), np.array(hc)

    def jac_c(self, y):
        """Jacobian of c as CSR with every structural entry stored."""
        X, R, V = self.split(y)
        N, nx, F, fd, dt = self.N, self.nx, self.F, self.fd, self.dt
        yv, yp, _ = self._vle(X)
        vals = {}
        for k in range(self.H):
            Xk, Rk, Vk = X[k], R[k], V[k]
            for i in range(nx):
                row = k * nx + i
                d = {}   # partials of rhs_i
                if i == 0:
                    d[self.ix(k, 0)] = -Vk
                    d[self.ix(k, 1)] = Vk * yp[k, 1]
                    d[self.iV(k)] = yv[k, 1] - Xk[0]
                elif i <= N:
                    lin = Rk if i <= fd else Rk + F
                    lout = Rk if i < fd else Rk + F
                    d[self.ix(k, i - 1)] = lin
                    d[self.ix(k, i)] = -lout - Vk * yp[k, i]
                    d[self.ix(k, i + 1)] = Vk * yp[k, i + 1]
                    d[self.iR(k)] = Xk[i - 1] - Xk[i]
                    d[self.iV(k)] = yv[k, i + 1] - yv[k, i]
                else:
                    d[self.ix(k, N)] = Rk + F
                    d[self.ix(k, N + 1)] = -Vk * yp[k, N + 1] - (Rk + F - Vk)
                    d[self.iR(k)] = Xk[N] - Xk[N + 1]
                    d[self.iV(k)] = -yv[k, N + 1] + Xk[N + 1]
                # c = x_k - x_{k-1} - dt * rhs
                out = {c: -dt * v for c, v in d.items()}
                out[self.ix(k, i)] = out.get(self.ix(k, i), 0.0) + 1.0
                if k > 0:
                    out[self.ix(k - 1, i)] = -1.0
                for c, v in out.items():
                    vals[(row, c)] = v
        for k in range(self.Hc, self.H):
            for j, idx in enumerate((self.iR, self.iV)):
                row = self.m_dyn + 2 * (k - self.Hc) + j
                vals[(row, idx(k - 1))] = -1.0
                vals[(row, idx(k))] = 1.0
        data = np.array([vals.get((r, c), 0.0) for r, c in zip(self.jc_rows, self.jc_cols)],
                        dtype=np.result_type(y, 1.0))
        return sp.csr_matrix((data, (self.jc_rows, self.jc_cols)), shape=(self.m_c, self.n))

    def jac_d(self, y):
        data = np.tile(np.array([1.0, -1.0, -1.0, 1.0]), self.H)
        return sp.csr_matrix((data, (self.jd_rows, self.jd_cols)), shape=(self.m_d, self.n))

    def hess(self, y, lam_c, lam_d):
        """Hessian of the Lagrangian f + lam_c^T c + lam_d^T d (full symmetric CSR)."""
        X, R, V = self.split(y)
        N, nx, dt, rho = self.N, self.nx, self.dt, self.rho
        _, yp, ypp = self._vle(X)
        Lam = np.asarray(lam_c)[:self.m_dyn].reshape(self.H, nx)   # the hold rows are linear
        vals = {}

        def add(i, j, v):
            key = (max(i, j), min(i, j))
            vals[key] = vals.get(key, 0.0) + v

        for k in range(self.H):
            Vk = V[k]
            lam = Lam[k]
            iR, iV = self.iR(k), self.iV(k)
            # objective
            add(self.ix(k, 0), self.ix(k, 0), 2.0)
            add(self.ix(k, N + 1), self.ix(k, N + 1), 2.0)
            wR = 2.0 * rho if k == self.H - 1 else 4.0 * rho
            add(iR, iR, wR)
            add(iV, iV, wR)
            if k > 0:
                add(iR, self.iR(k - 1), -2.0 * rho)
                add(iV, self.iV(k - 1), -2.0 * rho)
            # constraints: c_i = ... - dt * rhs_i, so weight is -dt * lam_i
            for i in range(nx):
                w = -dt * lam[i]
                if i == 0:
                    add(self.ix(k, 1), self.ix(k, 1), w * Vk * ypp[k, 1])
                    add(iV, self.ix(k, 1), w * yp[k, 1])
                    add(iV, self.ix(k, 0), -w)
                elif i <= N:
                    add(iR, self.ix(k, i - 1), w)
                    add(iR, self.ix(k, i), -w)
                    add(self.ix(k, i + 1), self.ix(k, i + 1), w * Vk * ypp[k, i + 1])
                    add(self.ix(k, i), self.ix(k, i), -w * Vk * ypp[k, i])
                    add(iV, self.ix(k, i + 1), w * yp[k, i + 1])
                    add(iV, self.ix(k, i), -w * yp[k, i])
                else:
                    add(iR, self.ix(k, N), w)
                    add(iR, self.ix(k, N + 1), -w)
                    add(self.ix(k, N + 1), self.ix(k, N + 1), -w * Vk * ypp[k, N + 1])
                    add(iV, self.ix(k, N + 1), w * (1.0 - yp[k, N + 1]))
        data = np.array([vals.get((r, c), 0.0) for r, c in zip(self.h_rows, self.h_cols)],
                        dtype=np.result_type(y, lam_c, 1.0))
        Wl = sp.csr_matrix((data, (self.h_rows, self.h_cols)), shape=(self.n, self.n))
        return (Wl + sp.triu(Wl.T, k=1)).tocsr()

    # ---- parameter derivatives (for sensitivities) ---------------------
    def parameter_derivatives(self, y):
        """Partial derivatives of the NLP functions with respect to each parameter
        group, as dense arrays: for group g, dc[g] (m_c x n_g), dd[g] (m_d x n_g),
        dgrad[g] (n x n_g) = d(grad f)/dp and df[g] (n_g,).
        Groups: x0 (nx), setpoint (xD*, xB*), zF (H), u_prev (2)."""
        X, R, V = self.split(y)
        nx, H, n = self.nx, self.H, self.n
        out = {}
        # x0 enters c_1 = x_1 - x0 - dt rhs(x_1, u_1)
        dc = np.zeros((self.m_c, nx))
        dc[:nx, :] = -np.eye(nx)
        out["x0"] = (dc, np.zeros((self.m_d, nx)), np.zeros((n, nx)), np.zeros(nx))
        # setpoints enter f only
        dg = np.zeros((n, 2))
        for k in range(H):
            dg[self.ix(k, 0), 0] = -2.0
            dg[self.ix(k, nx - 1), 1] = -2.0
        dfv = np.array([-2.0 * np.sum(X[:, 0] - self.xD_sp), -2.0 * np.sum(X[:, -1] - self.xB_sp)])
        out["setpoint"] = (np.zeros((self.m_c, 2)), np.zeros((self.m_d, 2)), dg, dfv)
        # feed composition zF_k enters rhs at the feed tray of stage k with weight F
        dc = np.zeros((self.m_c, H))
        for k in range(H):
            dc[k * nx + self.fd, k] = -self.dt * self.F
        out["zF"] = (dc, np.zeros((self.m_d, H)), np.zeros((n, H)), np.zeros(H))
        # u_prev enters the first move penalty
        dg = np.zeros((n, 2))
        dg[self.iR(0), 0] = -2.0 * self.rho
        dg[self.iV(0), 1] = -2.0 * self.rho
        dfv = np.array([-2.0 * self.rho * (R[0] - self.u_prev[0]), -2.0 * self.rho * (V[0] - self.u_prev[1])])
        out["u_prev"] = (np.zeros((self.m_c, 2)), np.zeros((self.m_d, 2)), dg, dfv)
        return out

    def u1_index(self):
        return [self.iR(0), self.iV(0)]

    # ---- starting point ------------------------------------------------
    def initial_guess(self):
        """Cold start: every stage holds the measured state and the last control."""
        y = np.empty(self.n)
        for k in range(self.H):
            y[self.ix(k, 0):self.ix(k, 0) + self.nx] = self.x0
            y[self.iR(k)] = self.u_prev[0]
            y[self.iV(k)] = self.u_prev[1]
        return y

    def u1(self, y):
        return np.array([y[self.iR(0)], y[self.iV(0)]])

    def x1(self, y):
        return np.array(y[self.ix(0, 0):self.ix(0, 0) + self.nx])
