"""Plant simulator for closed-loop studies (Algorithm 1 applies the first
control to the system and measures the next state).

The plant is the distillation column of the workload family (N trays plus
condenser and reboiler, constant molar overflow, relative volatility alpha,
feed on tray N/2, reflux R and boilup V) advanced by one implicit-Euler step
of dt, the discretization the controller's model uses, solved by Newton's
method on the host.  Giving the plant parameters other than the model's
(alpha, feed flow) is a plant-model mismatch: the controller then sees
measurements its predictions do not reproduce.  Host NumPy; not part of the
GPU path.
"""
from __future__ import annotations

import numpy as np


class DistillationPlant:
    def __init__(self, N, alpha, dt, F=1.0):
        self.N, self.alpha, self.dt, self.F = int(N), float(alpha), float(dt), float(F)
        self.nx = self.N + 2
        self.fd = self.N // 2

    def _vle(self, x):
        a = self.alpha
        g = 1.0 + (a - 1.0) * x
        return a * x / g, a / (g * g)

    def rate(self, x, R, V, zF):
        """dx/dt and its Jacobian d(dx/dt)/dx (tridiagonal, dense here)."""
        N, F, fd, nx = self.N, self.F, self.fd, self.nx
        y, yp = self._vle(x)
        r = np.empty(nx)
        J = np.zeros((nx, nx))
        r[0] = V * (y[1] - x[0])
        J[0, 0], J[0, 1] = -V, V * yp[1]
        for i in range(1, N + 1):
            lin = R if i <= fd else R + F
            lout = R if i < fd else R + F
            r[i] = lin * x[i - 1] - lout * x[i] + V * (y[i + 1] - y[i]) + (F * zF if i == fd else 0.0)
            J[i, i - 1] = lin
            J[i, i] = -lout - V * yp[i]
            J[i, i + 1] = V * yp[i + 1]
        r[N + 1] = (R + F) * x[N] - V * y[N + 1] - (R + F - V) * x[N + 1]
        J[N + 1, N], J[N + 1, N + 1] = R + F, -V * yp[N + 1] - (R + F - V)
        return r, J

    def step(self, x, u, zF=0.5, tol=1e-14, max_newton=30):
        """x(t + dt) with x+ - x - dt f(x+, u) = 0, from x+ = x."""
        x = np.asarray(x, dtype=np.float64)
        R, V = float(u[0]), float(u[1])
        z = x.copy()
        for _ in range(max_newton):
            f, J = self.rate(z, R, V, zF)
            res = z - x - self.dt * f
            if np.max(np.abs(res)) <= tol:
                break
            z = z - np.linalg.solve(np.eye(self.nx) - self.dt * J, res)
        return np.clip(z, 0.0, 1.0)
