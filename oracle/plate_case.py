"""The heated-plate case study of Section 4.2 (Table 2) as a transcribed OCP
(oracle side; test infrastructure only).

An aluminium plate on [-1, 1] x [-1, 1], n points per dimension (spacing
h = 2 / (n - 1) = L), heated through its left and bottom edges by the input Q:

    dT/dt = alpha (T_x1x1 + T_x2x2 - s)                      (interior points)
    T(-1, x2) = 4.1 Q^(1/3),  T(x1, -1) = Q^(1/2),  T(1, x2) = T(x1, 1) = T_b
    Q >= Q_lo
    min  integral over the horizon of
         [ integral over [-0.5, 0.5]^2 of (T - T_sp(t))^2 dx1 dx2 + rho Q^2 ] dt

with the loss term s as printed (5 q_loss^2) or as read (5 q_loss; see the
design notes).  Transcription: second-order central differences in space
(5-point stencil, the edge values as Dirichlet neighbours; the corner points
enter no stencil), backward Euler in time with the measured interior field as
the stage-0 parameter x0, the time integral by the backward rule (dt times the
sum over stages 1..H), the region integral by the trapezoid rule on the grid
points of [-0.5, 0.5]^2 (weights h^2 times 1/2 on the region's edges, 1/4 at
its corners).  T_sp(t) of each stage is the stage's trajectory value.

Scaling (fixed constants of the transcription, in place of the automatic
scaling of the paper's solvers): the decision variable for the input is
q = Q / q_scale, and every state row is divided by its diagonal coefficient
1 + 4 dt alpha / h^2, so rows read in temperature units.

Decision vector, stage-major, ns = (n - 2)^2 + 1 per stage: the interior
points with x1 fastest (node p = (j - 1)(n - 2) + (i - 1) at x1 = -1 + i h,
x2 = -1 + j h), then q.  Equality rows: one per interior point, node order.

All functions accept complex y for complex-step checks.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg.spsolve)

# Table 2 of the paper
TABLE2 = dict(alpha=230.0, L=0.1, Tb=50.0, n=21, rho=1e-8, q_loss=10.0)


class PlateCaseOCP:
    def __init__(self, H=12, dt=0.08, n=21, alpha=230.0, Tb=50.0, loss=50.0, rho=1e-8, Q_lo=50.0,
                 q_scale=1e4):
        self.H, self.dt, self.npts = int(H), float(dt), int(n)
        self.alpha, self.Tb, self.loss, self.rho = float(alpha), float(Tb), float(loss), float(rho)
        self.qs = float(q_scale)
        self.h = 2.0 / (self.npts - 1)
        self.g = self.npts - 2                    # interior points per dimension
        self.kap = self.dt * self.alpha / (self.h * self.h)
        self.rs = 1.0 / (1.0 + 4.0 * self.kap)    # row scale
        self.nx, self.nu = self.g * self.g, 1
        self.ns = self.nx + 1
        self.n = self.H * self.ns                 # decision variables
        self.m_c = self.H * self.nx
        self.m_d = 0
        self.rps = self.nx
        lb = np.full((self.H, self.ns), -np.inf)
        ub = np.full((self.H, self.ns), np.inf)
        lb[:, -1] = Q_lo / self.qs
        self.lb, self.ub = lb.reshape(-1), ub.reshape(-1)
        self.x0 = np.full(self.nx, self.Tb)
        self.traj = np.full(self.H, 58.0)
        self.u_prev = np.array([Q_lo / self.qs])
        # trapezoid weights of the tracking region on the interior grid
        x = -1.0 + self.h * np.arange(1, self.npts - 1)
        inside = np.abs(x) <= 0.5 + 1e-12
        edge = np.isclose(np.abs(x), 0.5)
        c = np.where(inside, np.where(edge, 0.5, 1.0), 0.0)
        self.weights = (self.h * self.h) * np.outer(c, c).reshape(-1)   # index (j, i) -> p
        self.coord = x
        self._build_patterns()

    # ---- parameters ----------------------------------------------------------
    def set_parameters(self, x0=None, traj=None, u_prev=None, **_):
        """u_prev in the decision variable's units (q = Q / q_scale)."""
        if x0 is not None:
            self.x0 = np.array(x0, dtype=np.float64).reshape(self.nx)
        if traj is not None:
            self.traj = np.array(traj, dtype=np.float64).reshape(self.H)
        if u_prev is not None:
            self.u_prev = np.array(u_prev, dtype=np.float64).reshape(1)

    def split(self, y):
        Y = y.reshape(self.H, self.ns)
        return Y[:, :self.nx], Y[:, self.nx]

    # ---- model --------------------------------------------------------------------
    def edges(self, Q):
        """(left, bottom) edge temperatures for the input Q (unscaled)."""
        return 4.1 * Q ** (1.0 / 3.0), Q ** 0.5

    def laplacian(self, T, Q):
        """5-point Laplacian of the interior field(s) T (..., g*g) with the
        Dirichlet edges of Q (...,)."""
        g, h = self.g, self.h
        T = T.reshape(T.shape[:-1] + (g, g))            # (..., j, i)
        left, bottom = self.edges(Q)
        P = np.zeros(T.shape[:-2] + (g + 2, g + 2), dtype=np.result_type(T, Q, 1.0))
        P[..., 1:-1, 1:-1] = T
        P[..., 1:-1, 0] = left[..., None]                # x1 = -1 (i = 0)
        P[..., 1:-1, -1] = self.Tb                       # x1 = 1
        P[..., 0, 1:-1] = bottom[..., None]              # x2 = -1 (j = 0)
        P[..., -1, 1:-1] = self.Tb                       # x2 = 1
        lap = (P[..., 1:-1, :-2] + P[..., 1:-1, 2:] + P[..., :-2, 1:-1] + P[..., 2:, 1:-1]
               - 4.0 * P[..., 1:-1, 1:-1]) / (h * h)
        return lap.reshape(T.shape[:-2] + (g * g,))

    def rhs(self, T, Q):
        return self.alpha * (self.laplacian(T, Q) - self.loss)

    # ---- NLP functions ------------------------------------------------------------------
    def f(self, y):
        T, q = self.split(y)
        E = T - self.traj[:, None]
        Q = self.qs * q
        return self.dt * (np.sum((E * E) @ self.weights) + self.rho * np.sum(Q * Q))

    def grad(self, y):
        T, q = self.split(y)
        G = np.zeros((self.H, self.ns), dtype=np.result_type(y, 1.0))
        G[:, :self.nx] = 2.0 * self.dt * (T - self.traj[:, None]) * self.weights
        G[:, self.nx] = 2.0 * self.dt * self.rho * self.qs * self.qs * q
        return G.reshape(-1)

    def cons_c(self, y):
        T, q = self.split(y)
        Tp = np.vstack([self.x0[None, :], T[:-1]])
        return (self.rs * (T - Tp - self.dt * self.rhs(T, self.qs * q))).reshape(-1)

    def cons_d(self, y):
        return np.zeros(0, dtype=np.result_type(y, 1.0))

    def _neighbours(self, p):
        g = self.g
        i, j = p % g, p // g
        nb = [p]
        if i > 0:
            nb.append(p - 1)
        if i < g - 1:
            nb.append(p + 1)
        if j > 0:
            nb.append(p - g)
        if j < g - 1:
            nb.append(p + g)
        return sorted(nb), i == 0, j == 0

    def _build_patterns(self):
        nx, ns = self.nx, self.ns
        jr, jc = [], []
        for k in range(self.H):
            for p in range(nx):
                nb, left, bottom = self._neighbours(p)
                cols = ([(k - 1) * ns + p] if k > 0 else []) + [k * ns + q for q in nb]
                if left or bottom:
                    cols.append(k * ns + nx)
                jr += [k * nx + p] * len(cols)
                jc += cols
        self.jc_rows, self.jc_cols = np.array(jr), np.array(jc)
        self.jd_rows = self.jd_cols = np.zeros(0, dtype=int)
        self.h_rows = np.arange(self.n)           # the Hessian of the Lagrangian is diagonal
        self.h_cols = np.arange(self.n)

    def _edge_derivatives(self, Q):
        """First and second derivatives of the left and bottom edge values in q."""
        s = self.qs
        d1 = (4.1 / 3.0 * Q ** (-2.0 / 3.0) * s, 0.5 * Q ** (-0.5) * s)
        d2 = (4.1 / 3.0 * (-2.0 / 3.0) * Q ** (-5.0 / 3.0) * s * s, 0.5 * (-0.5) * Q ** (-1.5) * s * s)
        return d1, d2

    def jac_c(self, y):
        T, q = self.split(y)
        nx, ns, kap, rs = self.nx, self.ns, self.kap, self.rs
        vals = {}
        for k in range(self.H):
            (dl, db), _ = self._edge_derivatives(self.qs * q[k])
            for p in range(nx):
                nb, left, bottom = self._neighbours(p)
                r = k * nx + p
                if k > 0:
                    vals[(r, (k - 1) * ns + p)] = -rs
                for qn in nb:
                    vals[(r, k * ns + qn)] = rs * (1.0 + 4.0 * kap) if qn == p else -rs * kap
                if left or bottom:
                    vals[(r, k * ns + nx)] = -rs * kap * ((dl if left else 0.0) + (db if bottom else 0.0))
        data = np.array([vals[(r, c)] for r, c in zip(self.jc_rows, self.jc_cols)])
        return sp.csr_matrix((data, (self.jc_rows, self.jc_cols)), shape=(self.m_c, self.n))

    def jac_d(self, y):
        return sp.csr_matrix((0, self.n))

    def hess(self, y, lam_c, lam_d):
        """Hessian of f + lam_c^T c: diagonal (the tracking weights on T; on q
        the rho term plus the edge curvature of the rows next to the heated
        edges)."""
        T, q = self.split(y)
        g, nx, ns, kap, rs = self.g, self.nx, self.ns, self.kap, self.rs
        Lam = np.asarray(lam_c).reshape(self.H, nx)
        diag = np.zeros((self.H, ns), dtype=np.result_type(y, lam_c, 1.0))
        diag[:, :nx] = 2.0 * self.dt * self.weights
        idx = np.arange(nx)
        on_left, on_bottom = idx % g == 0, idx < g
        for k in range(self.H):
            _, (d2l, d2b) = self._edge_derivatives(self.qs * q[k])
            s = np.sum(Lam[k, on_left]) * d2l + np.sum(Lam[k, on_bottom]) * d2b
            diag[k, nx] = 2.0 * self.dt * self.rho * self.qs * self.qs - rs * kap * s
        return sp.diags(diag.reshape(-1)).tocsr()

    def parameter_derivatives(self, y):
        """Groups: x0 (nx) enters the first stage's rows with coefficient -rs;
        traj (H): the tracked temperature of each stage, in the objective."""
        T, _ = self.split(y)
        nx, H, n, dt = self.nx, self.H, self.n, self.dt
        dc = np.zeros((self.m_c, nx))
        dc[:nx, :] = -self.rs * np.eye(nx)
        dg = np.zeros((n, H))
        for k in range(H):
            dg[k * self.ns:k * self.ns + nx, k] = -2.0 * dt * self.weights
        dfv = -2.0 * dt * ((T - self.traj[:, None]) @ self.weights)
        return {"x0": (dc, np.zeros((0, nx)), np.zeros((n, nx)), np.zeros(nx)),
                "traj": (np.zeros((self.m_c, H)), np.zeros((0, H)), dg, dfv)}

    def u1_index(self):
        return [self.nx]

    def initial_guess(self):
        """Cold start: every stage at the measured field and the last input."""
        return np.tile(np.concatenate([self.x0, self.u_prev]), self.H)

    def u1(self, y):
        return np.array([y[self.nx]])

    def x1(self, y):
        return np.array(y[:self.nx])

    def steady_state(self, Q):
        """Interior field with dT/dt = 0 for the input Q: the discrete Poisson
        problem lap_h T = s with the edges of Q, assembled as a sparse matrix
        (independently of `laplacian`) and solved directly."""
        g, h = self.g, self.h
        A = sp.lil_matrix((self.nx, self.nx))
        b = np.full(self.nx, self.loss * h * h)
        left, bottom = self.edges(np.float64(Q))
        for j in range(g):
            for i in range(g):
                p = j * g + i
                A[p, p] = -4.0
                for cond, q, val in ((i > 0, p - 1, left), (i < g - 1, p + 1, self.Tb), (j > 0, p - g, bottom),
                                     (j < g - 1, p + g, self.Tb)):
                    if cond:
                        A[p, q] = 1.0
                    else:
                        b[p] -= val
        return sp.linalg.spsolve(A.tocsr(), b)
