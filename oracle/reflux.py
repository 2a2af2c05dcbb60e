"""The distillation case study of Section 4.1 as a transcribed OCP (oracle side;
test infrastructure only).

A column of N trays (tray 1 the condenser, tray N the reboiler) with the feed
on tray N_f, fixed distillate flow D, controlled by the reflux ratio u.  The
algebraic quantities of the paper's formulation stay variables with their own
equality rows, as written there:

    y_i = alpha x_i / (1 + (alpha - 1) x_i)       (vapour-liquid equilibrium)
    L = u D,   V = L + D,   S = L + F             (liquid, vapour, stripping flows)

    dx_1/dt   = V (y_2 - x_1) / A_c
    dx_j/dt   = (L (x_{j-1} - x_j) - V (y_j - y_{j+1})) / A_t,            j = 2 .. N_f - 1
    dx_Nf/dt  = (F x_f + L x_{Nf-1} - S x_Nf - V (y_Nf - y_{Nf+1})) / A_t
    dx_k/dt   = (S (x_{k-1} - x_k) - V (y_k - y_{k+1})) / A_t,            k = N_f + 1 .. N - 1
    dx_N/dt   = (S x_{N-1} - (F - D) x_N - V y_N) / A_r

(the paper's range for the stripping trays reads N_f + 1 .. N, which would
need y_{N+1}; the reboiler has its own equation, so the range ends at N - 1).
Objective: the integral of (x_1 - xbar)^2 + w_u (u - ubar)^2 over the
horizon, by the backward-difference rule: dt times the sum over stages 1..H.
Bounds: x, y in [0, 1]; u in [1, 5]; L, V, S in [0, 10].  Backward Euler,
x at stage 0 the measured parameter x0 (the initial algebraic values do not
enter the backward-difference transcription).

Decision vector, stage-major, ns = 2 N + 4 per stage:
    [x_1 .. x_N, u, y_1 .. y_N, L, V, S]
Equality rows, stage-major, 2 N + 3 per stage: N dynamics rows (tray order),
N equilibrium rows y_i - phi(x_i), then L - u D, V - L - D, S - L - F.

All functions accept complex y for complex-step checks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Table 1 of the paper
TABLE1 = dict(N=32, Nf=17, D=0.2, F=0.4, alpha=1.6, xbar=0.8958, ubar=2.51459, xf=0.5, Ac=0.5, At=0.25,
              Ar=1.0)


class RefluxColumnOCP:
    def __init__(self, H, dt=2.0, N=32, Nf=17, D=0.2, F=0.4, alpha=1.6, xbar=0.8958, ubar=2.51459, xf=0.5,
                 Ac=0.5, At=0.25, Ar=1.0, w_u=0.1, u_lo=1.0, u_hi=5.0, flow_hi=10.0):
        self.N, self.Nf, self.H, self.dt = int(N), int(Nf), int(H), float(dt)
        self.D, self.F, self.alpha, self.xf = float(D), float(F), float(alpha), float(xf)
        self.Ac, self.At, self.Ar, self.w_u = float(Ac), float(At), float(Ar), float(w_u)
        self.xbar, self.ubar = float(xbar), float(ubar)
        self.nx, self.nu = self.N, 1
        self.ns = 2 * self.N + 4
        self.rps = 2 * self.N + 3
        self.n = self.H * self.ns
        self.m_c = self.H * self.rps
        self.m_d = 0
        lb = np.zeros((self.H, self.ns))
        ub = np.ones((self.H, self.ns))
        lb[:, self.iu] , ub[:, self.iu] = u_lo, u_hi
        lb[:, self.iL:], ub[:, self.iL:] = 0.0, flow_hi
        self.lb, self.ub = lb.reshape(-1), ub.reshape(-1)
        self.x0 = self.steady_state(2.0)
        self.u_prev = np.array([2.0])
        self._build_patterns()

    # ---- index helpers (within a stage) --------------------------------------
    @property
    def iu(self):
        return self.N

    @property
    def iL(self):
        return 2 * self.N + 1

    def ix(self, i):          # tray i (1-based)
        return i - 1

    def iy(self, i):
        return self.N + i

    def set_parameters(self, x0=None, setpoint=None, u_prev=None, **_):
        if x0 is not None:
            self.x0 = np.array(x0, dtype=np.float64).reshape(self.N)
        if setpoint is not None:
            self.xbar, self.ubar = float(setpoint[0]), float(setpoint[1])
        if u_prev is not None:
            self.u_prev = np.array(u_prev, dtype=np.float64).reshape(1)

    def split(self, y):
        Y = y.reshape(self.H, self.ns)
        N = self.N
        return Y[:, :N], Y[:, N], Y[:, N + 1:2 * N + 1], Y[:, 2 * N + 1], Y[:, 2 * N + 2], Y[:, 2 * N + 3]

    def _phi(self, x):
        a = self.alpha
        g = 1.0 + (a - 1.0) * x
        return a * x / g, a / g ** 2, -2.0 * a * (a - 1.0) / g ** 3

    # ---- model right-hand side (also used for the steady state) --------------
    def rhs(self, X, Yv, L, V, S):
        """dx/dt per stage: X, Yv (..., N); L, V, S (...,)."""
        N, Nf, F, D, xf = self.N, self.Nf, self.F, self.D, self.xf
        L, V, S = (np.asarray(v)[..., None] for v in (L, V, S))
        out = np.zeros(np.broadcast(X, Yv, L).shape, dtype=np.result_type(X, Yv, L, 1.0))
        out[..., 0] = V[..., 0] * (Yv[..., 1] - X[..., 0]) / self.Ac
        for j in range(2, Nf):
            out[..., j - 1] = (L[..., 0] * (X[..., j - 2] - X[..., j - 1])
                               - V[..., 0] * (Yv[..., j - 1] - Yv[..., j])) / self.At
        j = Nf
        out[..., j - 1] = (F * xf + L[..., 0] * X[..., j - 2] - S[..., 0] * X[..., j - 1]
                           - V[..., 0] * (Yv[..., j - 1] - Yv[..., j])) / self.At
        for k in range(Nf + 1, N):
            out[..., k - 1] = (S[..., 0] * (X[..., k - 2] - X[..., k - 1])
                               - V[..., 0] * (Yv[..., k - 1] - Yv[..., k])) / self.At
        out[..., N - 1] = (S[..., 0] * X[..., N - 2] - (F - D) * X[..., N - 1] - V[..., 0] * Yv[..., N - 1]) / self.Ar
        return out

    def flows(self, u):
        L = u * self.D
        return L, L + self.D, L + self.F

    def steady_state(self, u, x_guess=None, iters=50):
        """Tray compositions with dx/dt = 0 at constant reflux ratio u (Newton
        on the N balances with y = phi(x), by dense finite-difference-free
        complex-step Jacobians)."""
        L, V, S = self.flows(u)
        x = np.linspace(0.9, 0.1, self.N) if x_guess is None else np.array(x_guess, float)

        def f(xx):
            return self.rhs(xx, self._phi(xx)[0], L, V, S)

        for _ in range(iters):
            r = f(x)
            if np.max(np.abs(r)) < 1e-15:
                break
            J = np.empty((self.N, self.N))
            for c in range(self.N):
                e = np.zeros(self.N, dtype=complex)
                e[c] = 1e-30j
                J[:, c] = np.imag(f(x + e)) / 1e-30
            x = x - np.linalg.solve(J, r)
        return x

    # ---- NLP functions -------------------------------------------------------
    def f(self, y):
        X, U, *_ = self.split(y)
        return self.dt * (np.sum((X[:, 0] - self.xbar) ** 2) + self.w_u * np.sum((U - self.ubar) ** 2))

    def grad(self, y):
        X, U, *_ = self.split(y)
        G = np.zeros((self.H, self.ns), dtype=np.result_type(y, 1.0))
        G[:, 0] = 2.0 * self.dt * (X[:, 0] - self.xbar)
        G[:, self.iu] = 2.0 * self.dt * self.w_u * (U - self.ubar)
        return G.reshape(-1)

    def cons_c(self, y):
        X, U, Yv, L, V, S = self.split(y)
        Xp = np.vstack([self.x0[None, :], X[:-1]])
        dyn = X - Xp - self.dt * self.rhs(X, Yv, L, V, S)
        vle = Yv - self._phi(X)[0]
        fl = np.stack([L - U * self.D, V - L - self.D, S - L - self.F], axis=1)
        return np.concatenate([dyn, vle, fl], axis=1).reshape(-1)

    def cons_d(self, y):
        return np.zeros(0, dtype=np.result_type(y, 1.0))

    # ---- patterns and derivative values ----------------------------------------
    def _dyn_partials(self, i, Xk, Yk, Lk, Vk, Sk):
        """{stage-local column: d f_i / d column} for the dynamics of tray i."""
        N, Nf, F, D = self.N, self.Nf, self.F, self.D
        ix, iy, iL = self.ix, self.iy, self.iL
        iV, iS = iL + 1, iL + 2
        if i == 1:
            return {ix(1): -Vk / self.Ac, iy(2): Vk / self.Ac, iV: (Yk[1] - Xk[0]) / self.Ac}
        if i < Nf:
            return {ix(i - 1): Lk / self.At, ix(i): -Lk / self.At, iy(i): -Vk / self.At, iy(i + 1): Vk / self.At,
                    iL: (Xk[i - 2] - Xk[i - 1]) / self.At, iV: -(Yk[i - 1] - Yk[i]) / self.At}
        if i == Nf:
            return {ix(i - 1): Lk / self.At, ix(i): -Sk / self.At, iy(i): -Vk / self.At, iy(i + 1): Vk / self.At,
                    iL: Xk[i - 2] / self.At, iV: -(Yk[i - 1] - Yk[i]) / self.At, iS: -Xk[i - 1] / self.At}
        if i < N:
            return {ix(i - 1): Sk / self.At, ix(i): -Sk / self.At, iy(i): -Vk / self.At, iy(i + 1): Vk / self.At,
                    iV: -(Yk[i - 1] - Yk[i]) / self.At, iS: (Xk[i - 2] - Xk[i - 1]) / self.At}
        return {ix(N - 1): Sk / self.Ar, ix(N): -(F - D) / self.Ar, iy(N): -Vk / self.Ar, iV: -Yk[N - 1] / self.Ar,
                iS: Xk[N - 2] / self.Ar}

    def _build_patterns(self):
        N, H, ns, rps = self.N, self.H, self.ns, self.rps
        z = np.zeros(N)
        rows, cols = [], []
        for k in range(H):
            for i in range(1, N + 1):
                cs = set(self._dyn_partials(i, z, z, 0.0, 0.0, 0.0)) | {self.ix(i)}
                row = k * rps + i - 1
                if k > 0:
                    rows.append(row)
                    cols.append((k - 1) * ns + self.ix(i))
                for c in sorted(cs):
                    rows.append(row)
                    cols.append(k * ns + c)
            for i in range(1, N + 1):
                row = k * rps + N + i - 1
                rows += [row, row]
                cols += [k * ns + self.ix(i), k * ns + self.iy(i)]
            iL = self.iL
            for r, (a, b) in enumerate(((self.iu, iL), (iL, iL + 1), (iL, iL + 2))):
                row = k * rps + 2 * N + r
                rows += [row, row]
                cols += [k * ns + a, k * ns + b]
        self.jc_rows, self.jc_cols = np.array(rows), np.array(cols)
        self.jd_rows = self.jd_cols = np.zeros(0, dtype=int)
        # Hessian of the Lagrangian, lower triangle: x diagonal, u diagonal,
        # (L, x_j) j < N_f, (S, x_j) N_f <= j < N, (V, x_1), (V, y_j) j >= 2
        hr, hc = [], []
        for k in range(H):
            o = k * ns
            for i in range(1, N + 1):
                hr.append(o + self.ix(i)); hc.append(o + self.ix(i))
            hr.append(o + self.iu); hc.append(o + self.iu)
            for j in range(1, self.Nf):
                hr.append(o + self.iL); hc.append(o + self.ix(j))
            for j in range(self.Nf, N):
                hr.append(o + self.iL + 2); hc.append(o + self.ix(j))
            hr.append(o + self.iL + 1); hc.append(o + self.ix(1))
            for j in range(2, N + 1):
                hr.append(o + self.iL + 1); hc.append(o + self.iy(j))
        self.h_rows, self.h_cols = np.array(hr), np.array(hc)

    def jac_c(self, y):
        X, U, Yv, L, V, S = self.split(y)
        N, H, ns, rps, dt = self.N, self.H, self.ns, self.rps, self.dt
        vals = {}
        _, dphi, _ = self._phi(X)
        for k in range(H):
            for i in range(1, N + 1):
                row = k * rps + i - 1
                for c, v in self._dyn_partials(i, X[k], Yv[k], L[k], V[k], S[k]).items():
                    vals[(row, k * ns + c)] = -dt * v
                vals[(row, k * ns + self.ix(i))] = vals.get((row, k * ns + self.ix(i)), 0.0) + 1.0
                if k > 0:
                    vals[(row, (k - 1) * ns + self.ix(i))] = -1.0
                row = k * rps + N + i - 1
                vals[(row, k * ns + self.ix(i))] = -dphi[k, i - 1]
                vals[(row, k * ns + self.iy(i))] = 1.0
            iL = self.iL
            for r, ((a, va), (b, vb)) in enumerate((((self.iu, -self.D), (iL, 1.0)), ((iL, -1.0), (iL + 1, 1.0)),
                                                   ((iL, -1.0), (iL + 2, 1.0)))):
                row = k * rps + 2 * N + r
                vals[(row, k * ns + a)] = va
                vals[(row, k * ns + b)] = vb
        data = np.array([vals.get((r, c), 0.0) for r, c in zip(self.jc_rows, self.jc_cols)],
                        dtype=np.result_type(y, 1.0))
        return sp.csr_matrix((data, (self.jc_rows, self.jc_cols)), shape=(self.m_c, self.n))

    def jac_d(self, y):
        return sp.csr_matrix((self.m_d, self.n))

    def hess(self, y, lam_c, lam_d):
        """Hessian of f + lam_c^T c (full symmetric CSR)."""
        X, U, Yv, L, V, S = self.split(y)
        N, Nf, H, ns, rps, dt = self.N, self.Nf, self.H, self.ns, self.rps, self.dt
        _, _, ddphi = self._phi(X)
        Lam = np.asarray(lam_c).reshape(H, rps)
        vals = {}

        def add(i, j, v):
            key = (max(i, j), min(i, j))
            vals[key] = vals.get(key, 0.0) + v

        for k in range(H):
            o = k * ns
            ld = Lam[k, :N]          # dynamics rows: c = x - x_prev - dt f, second derivatives -dt d2f
            lv = Lam[k, N:2 * N]     # equilibrium rows: c = y - phi(x)
            ix, iy = (lambda i: o + self.ix(i)), (lambda i: o + self.iy(i))
            iL, iV, iS = o + self.iL, o + self.iL + 1, o + self.iL + 2
            add(ix(1), ix(1), 2.0 * dt)
            add(o + self.iu, o + self.iu, 2.0 * dt * self.w_u)
            for i in range(1, N + 1):
                add(ix(i), ix(i), -lv[i - 1] * ddphi[k, i - 1])
            w = lambda i, A: -dt * ld[i - 1] / A   # noqa: E731
            add(iV, iy(2), w(1, self.Ac))
            add(iV, ix(1), -w(1, self.Ac))
            for i in range(2, Nf):
                add(iL, ix(i - 1), w(i, self.At)); add(iL, ix(i), -w(i, self.At))
                add(iV, iy(i), -w(i, self.At)); add(iV, iy(i + 1), w(i, self.At))
            add(iL, ix(Nf - 1), w(Nf, self.At)); add(iS, ix(Nf), -w(Nf, self.At))
            add(iV, iy(Nf), -w(Nf, self.At)); add(iV, iy(Nf + 1), w(Nf, self.At))
            for i in range(Nf + 1, N):
                add(iS, ix(i - 1), w(i, self.At)); add(iS, ix(i), -w(i, self.At))
                add(iV, iy(i), -w(i, self.At)); add(iV, iy(i + 1), w(i, self.At))
            add(iS, ix(N - 1), w(N, self.Ar)); add(iV, iy(N), -w(N, self.Ar))
        data = np.array([vals.get((r, c), 0.0) for r, c in zip(self.h_rows, self.h_cols)],
                        dtype=np.result_type(y, lam_c, 1.0))
        Wl = sp.csr_matrix((data, (self.h_rows, self.h_cols)), shape=(self.n, self.n))
        return (Wl + sp.triu(Wl.T, k=1)).tocsr()

    # ---- parameter derivatives (sensitivities) -------------------------------
    def parameter_derivatives(self, y):
        """Groups: x0 (N), setpoint (xbar, ubar), u_prev (1: enters nothing)."""
        X, U, *_ = self.split(y)
        N, H, n, dt = self.N, self.H, self.n, self.dt
        out = {}
        dc = np.zeros((self.m_c, N))
        dc[:N, :] = -np.eye(N)
        out["x0"] = (dc, np.zeros((0, N)), np.zeros((n, N)), np.zeros(N))
        dg = np.zeros((n, 2))
        for k in range(H):
            dg[k * self.ns + self.ix(1), 0] = -2.0 * dt
            dg[k * self.ns + self.iu, 1] = -2.0 * dt * self.w_u
        dfv = np.array([-2.0 * dt * np.sum(X[:, 0] - self.xbar), -2.0 * dt * self.w_u * np.sum(U - self.ubar)])
        out["setpoint"] = (np.zeros((self.m_c, 2)), np.zeros((0, 2)), dg, dfv)
        out["u_prev"] = (np.zeros((self.m_c, 1)), np.zeros((0, 1)), np.zeros((n, 1)), np.zeros(1))
        return out

    def u1_index(self):
        return [self.iu]

    def initial_guess(self):
        """Cold start: every stage at the measured trays, the last reflux ratio,
        the equilibrium vapour and the flows it gives."""
        y = np.empty((self.H, self.ns))
        u = float(self.u_prev[0])
        L, V, S = self.flows(u)
        y[:, :self.N] = self.x0
        y[:, self.iu] = u
        y[:, self.N + 1:2 * self.N + 1] = self._phi(self.x0)[0]
        y[:, self.iL:] = (L, V, S)
        return y.reshape(-1)

    def u1(self, y):
        return np.array([y[self.iu]])

    def x1(self, y):
        return np.array(y[:self.N])
