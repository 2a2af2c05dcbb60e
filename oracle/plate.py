"""Transcribed heated-plate OCP (oracle side).

A stand-in of the Section 4.2 family (a plate whose temperature field follows
a nonlinear heat equation, transcribed by central differences in space and
backward differences in time, controlled from its edges), in the form the
benchmark workloads fix:

* G x G interior nodes at (a h, b h), h = 1 / (G + 1); node p = b G + a.
* Dirichlet heaters: the ghost node beyond an edge takes the value of its
  heater segment.  Edges in the order bottom (b = -1), right (a = G), top
  (b = G), left (a = -1); each edge has 4 segments of G / 4 ghost nodes along
  increasing coordinate; segment s = 4 edge + (coordinate // (G / 4)).
* Conductivity k(T) = 1 + sigma T, face average between neighbours, so the
  flux from q into p is [(T_q - T_p) + (sigma / 2)(T_q^2 - T_p^2)] / h^2 and
  dT_p/dt = sum over the 4 neighbours q of that flux.
* Transcription (stages k = 1..H, T at stage 0 is the parameter x0):
  c_{k,p} = T_{k,p} - T_{k-1,p} - dt * dT_p/dt (T_k, u_k) = 0.
* Objective: sum_k sum_p (T_{k,p} - T*_p)^2 (T* is the setpoint field): the
  tracking integral without its constant area weight h^2, which leaves the
  minimiser unchanged and keeps the objective curvature of order one next to
  the large lifted penalty weights of the condensed matrix.
* Bounds: T <= t_hi (upper only), c_lo <= u <= c_hi.  No other inequalities.

Decision vector y is stage-major: stage k occupies y[k ns:(k+1) ns] with
ns = G^2 + 16, laid out [T (G^2, node order), u (16)].

All functions accept complex y so derivatives can be checked by complex step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg.spsolve)

N_SEGMENTS = 16


def ghost_segments(G):
    """For each interior node p, the list of (segment) of its ghost neighbours."""
    if G % 4:
        raise ValueError("the grid size must be a multiple of 4 (4 heater segments per edge)")
    q = G // 4
    out = [[] for _ in range(G * G)]
    for b in range(G):
        for a in range(G):
            p = b * G + a
            if b == 0:
                out[p].append(0 * 4 + a // q)
            if a == G - 1:
                out[p].append(1 * 4 + b // q)
            if b == G - 1:
                out[p].append(2 * 4 + a // q)
            if a == 0:
                out[p].append(3 * 4 + b // q)
    return out


def interior_neighbours(G):
    out = []
    for b in range(G):
        for a in range(G):
            nb = []
            if b > 0:
                nb.append((b - 1) * G + a)
            if a > 0:
                nb.append(b * G + a - 1)
            if a < G - 1:
                nb.append(b * G + a + 1)
            if b < G - 1:
                nb.append((b + 1) * G + a)
            out.append(nb)
    return out


class PlateOCP:
    def __init__(self, G, H, dt, sigma=0.1, t_hi=1.5, c_lo=0.0, c_hi=1.0):
        self.G, self.H, self.dt = int(G), int(H), float(dt)
        self.sigma = float(sigma)
        self.kap = 0.5 * self.sigma
        self.h = 1.0 / (self.G + 1)
        self.nx = self.G * self.G
        self.nu = N_SEGMENTS
        self.ns = self.nx + self.nu
        self.n = self.H * self.ns
        self.m_c = self.H * self.nx
        self.m_d = 0
        self.ghosts = ghost_segments(self.G)
        self.nbrs = interior_neighbours(self.G)
        lb = np.empty(self.n)
        ub = np.empty(self.n)
        for k in range(self.H):
            o = k * self.ns
            lb[o:o + self.nx], ub[o:o + self.nx] = -np.inf, t_hi
            lb[o + self.nx:o + self.ns], ub[o + self.nx:o + self.ns] = c_lo, c_hi
        self.lb, self.ub = lb, ub
        self.x0 = np.zeros(self.nx)
        self.target = np.zeros(self.nx)
        self.u_prev = np.full(self.nu, 0.5)
        self._build_patterns()

    @classmethod
    def from_workload(cls, w, **over):
        m = cls(w.G, w.H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi, **over)
        m.set_parameters(x0=w.T0, target=w.target)
        return m

    def set_parameters(self, x0=None, target=None, u_prev=None, setpoint=None):
        if x0 is not None:
            self.x0 = np.array(x0, dtype=np.float64).reshape(self.nx)
        if setpoint is not None:
            target = setpoint
        if target is not None:
            self.target = np.array(target, dtype=np.float64).reshape(self.nx)
        if u_prev is not None:
            self.u_prev = np.array(u_prev, dtype=np.float64).reshape(self.nu)

    # ---- index helpers -------------------------------------------------
    def iT(self, k, p):
        return k * self.ns + p

    def iu(self, k, s):
        return k * self.ns + self.nx + s

    def split(self, y):
        Y = y.reshape(self.H, self.ns)
        return Y[:, :self.nx], Y[:, self.nx:]

    # ---- model right-hand side ----------------------------------------
    def rhs(self, T, U):
        """dT/dt for every stage: T (H, nx), U (H, nu) -> (H, nx)."""
        kap, h2 = self.kap, self.h * self.h
        out = np.zeros_like(T + 0.0 * U[:, :1])
        for p in range(self.nx):
            Tp = T[:, p]
            acc = 0.0 * Tp
            for q in self.nbrs[p]:
                Tq = T[:, q]
                acc = acc + (Tq - Tp) + kap * (Tq * Tq - Tp * Tp)
            for s in self.ghosts[p]:
                Us = U[:, s]
                acc = acc + (Us - Tp) + kap * (Us * Us - Tp * Tp)
            out[:, p] = acc / h2
        return out

    # ---- NLP functions -------------------------------------------------
    def f(self, y):
        T, _ = self.split(y)
        return np.sum((T - self.target[None, :]) ** 2)

    def grad(self, y):
        T, _ = self.split(y)
        G = np.zeros((self.H, self.ns), dtype=np.result_type(y, 1.0))
        G[:, :self.nx] = 2.0 * (T - self.target[None, :])
        return G.reshape(-1)

    def cons_c(self, y):
        T, U = self.split(y)
        Tp = np.vstack([self.x0[None, :], T[:-1]])
        return (T - Tp - self.dt * self.rhs(T, U)).reshape(-1)

    def cons_d(self, y):
        return np.zeros(0, dtype=np.result_type(y, 1.0))

    # ---- structural patterns and derivative values --------------------
    def _build_patterns(self):
        jr, jc = [], []
        for k in range(self.H):
            for p in range(self.nx):
                row = k * self.nx + p
                cols = set()
                if k > 0:
                    cols.add(self.iT(k - 1, p))
                cols.add(self.iT(k, p))
                for q in self.nbrs[p]:
                    cols.add(self.iT(k, q))
                for s in self.ghosts[p]:
                    cols.add(self.iu(k, s))
                for c in sorted(cols):
                    jr.append(row)
                    jc.append(c)
        self.jc_rows, self.jc_cols = np.array(jr), np.array(jc)
        self.jd_rows = self.jd_cols = np.zeros(0, dtype=int)
        idx = np.arange(self.n)
        self.h_rows, self.h_cols = idx.copy(), idx.copy()   # the Hessian is diagonal

    def jac_c(self, y):
        T, U = self.split(y)
        kap, h2, dt = self.kap, self.h * self.h, self.dt
        vals = {}
        for k in range(self.H):
            for p in range(self.nx):
                row = k * self.nx + p
                deg = len(self.nbrs[p]) + len(self.ghosts[p])
                vals[(row, self.iT(k, p))] = 1.0 + dt * deg * (1.0 + 2.0 * kap * T[k, p]) / h2
                if k > 0:
                    vals[(row, self.iT(k - 1, p))] = -1.0
                for q in self.nbrs[p]:
                    vals[(row, self.iT(k, q))] = -dt * (1.0 + 2.0 * kap * T[k, q]) / h2
                for s in self.ghosts[p]:
                    vals[(row, self.iu(k, s))] = -dt * (1.0 + 2.0 * kap * U[k, s]) / h2
        data = np.array([vals[(r, c)] for r, c in zip(self.jc_rows, self.jc_cols)], dtype=np.result_type(y, 1.0))
        return sp.csr_matrix((data, (self.jc_rows, self.jc_cols)), shape=(self.m_c, self.n))

    def jac_d(self, y):
        return sp.csr_matrix((0, self.n))

    def hess(self, y, lam_c, lam_d):
        """Hessian of the Lagrangian f + lam_c^T c (diagonal; full CSR)."""
        kap, h2, dt = self.kap, self.h * self.h, self.dt
        Lam = np.asarray(lam_c).reshape(self.H, self.nx)
        d = np.zeros((self.H, self.ns), dtype=np.result_type(y, lam_c, 1.0))
        d[:, :self.nx] = 2.0
        for k in range(self.H):
            for p in range(self.nx):
                deg = len(self.nbrs[p]) + len(self.ghosts[p])
                # c_{k,p} holds -dt/h^2 * (-kap T_p^2) once per neighbour
                d[k, p] += Lam[k, p] * 2.0 * kap * dt * deg / h2
                # c_{k,q} holds -dt/h^2 * kap T_p^2 for each interior neighbour q of p
                for q in self.nbrs[p]:
                    d[k, p] -= Lam[k, q] * 2.0 * kap * dt / h2
                for s in self.ghosts[p]:
                    d[k, self.nx + s] -= Lam[k, p] * 2.0 * kap * dt / h2
        return sp.diags(d.reshape(-1)).tocsr()

    # ---- parameter derivatives (for sensitivities) ---------------------
    def parameter_derivatives(self, y):
        """Groups: x0 (nx) enters c_1 = T_1 - x0 - dt rhs; setpoint (the target
        field, nx) enters f."""
        T, _ = self.split(y)
        nx, n = self.nx, self.n
        dc = np.zeros((self.m_c, nx))
        dc[:nx, :] = -np.eye(nx)
        out = {"x0": (dc, np.zeros((0, nx)), np.zeros((n, nx)), np.zeros(nx))}
        dg = np.zeros((n, nx))
        for k in range(self.H):
            dg[k * self.ns:k * self.ns + nx, :] = -2.0 * np.eye(nx)
        dfv = -2.0 * np.sum(T - self.target[None, :], axis=0)
        out["setpoint"] = (np.zeros((self.m_c, nx)), np.zeros((0, nx)), dg, dfv)
        return out

    def u1_index(self):
        return list(range(self.nx, self.ns))

    # ---- starting point ------------------------------------------------
    def initial_guess(self):
        """Cold start: every stage holds the measured field and the last control."""
        y = np.empty(self.n)
        for k in range(self.H):
            y[k * self.ns:k * self.ns + self.nx] = self.x0
            y[k * self.ns + self.nx:(k + 1) * self.ns] = self.u_prev
        return y

    def u1(self, y):
        return np.array(y[self.nx:self.ns])

    def x1(self, y):
        return np.array(y[:self.nx])

    # ---- simulation (for pins and the closed loop) ----------------------
    def step(self, x, u, tol=1e-13, max_newton=50):
        """One implicit-Euler step of the plant: solve c(T) = 0 for T given the
        previous field x and controls u, by Newton's method."""
        T = np.array(x, dtype=np.float64)
        one = PlateOCP(self.G, 1, self.dt, sigma=self.sigma)
        one.set_parameters(x0=x)
        for _ in range(max_newton):
            y = np.concatenate([T, u])
            r = one.cons_c(y)
            if np.max(np.abs(r)) <= tol:
                break
            J = one.jac_c(y).tocsc()[:, :self.nx]
            T = T - sp.linalg.spsolve(J, r)
        return T
