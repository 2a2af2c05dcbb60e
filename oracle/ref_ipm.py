"""Reference route (test infrastructure only): a plain primal-dual
interior-point method on the transcribed NLP of eq. (6) as posed, without the
lifting of eq. (16).

    min f(y)  s.t.  c(y) = 0,  d(y) <= 0,  lb <= y <= ub

Inequalities get slacks, d(y) + s = 0 with s >= 0; bounds and slacks are
barrier terms.  Each Newton step solves the unreduced augmented system

    [ W + Sigma_y + dw I   J_c^T     J_d^T        ] [dy     ]
    [ J_c                  -dc I     0            ] [dlambda]  = -[...]
    [ J_d                  0         -Sigma_s^{-1}] [dnu    ]

densely with LDL^T (scipy.linalg.ldl); its inertia, read from the block
diagonal D, must be (n, m_c + m_d, 0), otherwise dw grows (and dc > 0 is added
for a zero eigenvalue).  Separate primal and dual step lengths from the
fraction-to-boundary rule; backtracking on the l1 merit
phi_mu + nu (|c|_1 + |d + s|_1).  Monotone barrier decrease; stop at
E_0 <= tol.  This is the textbook method the lifted variant approximates, so
its solution is the KKT point of the original problem that the lifted method
(oracle and GPU) must reproduce within O(gamma + mu_final).  Dense, so meant for
the small workloads (n of a few hundred to a few thousand).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla


@dataclass
class RefResult:
    status: int          # 0 converged, 1 iteration limit, 2 line-search failure, 3 regularization failure
    iters: int
    y: np.ndarray
    lam: np.ndarray      # equality multipliers (Lagrangian f + lam^T c + nu^T d)
    nu: np.ndarray       # inequality multipliers
    zL: np.ndarray
    zU: np.ndarray
    E0: float
    mu: float


def _ftb(v, dv, tau):
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))


def _inertia(D):
    """(positive, negative, zero) eigenvalue counts of the block diagonal D."""
    pos = neg = zero = 0
    i, n = 0, D.shape[0]
    while i < n:
        if i + 1 < n and D[i + 1, i] != 0.0:
            ev = np.linalg.eigvalsh(D[i:i + 2, i:i + 2])
            i += 2
        else:
            ev = [D[i, i]]
            i += 1
        for e in ev:
            if e > 0:
                pos += 1
            elif e < 0:
                neg += 1
            else:
                zero += 1
    return pos, neg, zero


class ReferenceIPM:
    def __init__(self, nlp, tol=1e-10, mu0=0.1, mu_min=1e-12, max_iter=300):
        self.nlp, self.tol, self.mu0, self.mu_min, self.max_iter = nlp, tol, mu0, mu_min, max_iter
        self.hasL, self.hasU = np.isfinite(nlp.lb), np.isfinite(nlp.ub)

    def _gaps(self, y):
        return (np.where(self.hasL, y - self.nlp.lb, 1.0), np.where(self.hasU, self.nlp.ub - y, 1.0))

    def _errors(self, y, s, lam, nu, zs, zL, zU, mu):
        nlp = self.nlp
        gL, gU = self._gaps(y)
        r = nlp.grad(y) + nlp.jac_c(y).T @ lam - np.where(self.hasL, zL, 0.0) + np.where(self.hasU, zU, 0.0)
        e = [np.max(np.abs(r)), np.max(np.abs(nlp.cons_c(y)))]
        if nlp.m_d:
            r = r + nlp.jac_d(y).T @ nu
            e[0] = np.max(np.abs(r))
            e += [np.max(np.abs(nlp.cons_d(y) + s)), np.max(np.abs(nu - zs)), np.max(np.abs(s * zs - mu))]
        if np.any(self.hasL):
            e.append(np.max(np.abs((gL * zL - mu)[self.hasL])))
        if np.any(self.hasU):
            e.append(np.max(np.abs((gU * zU - mu)[self.hasU])))
        return float(max(e))

    def _phi(self, y, s, mu, pen):
        nlp = self.nlp
        gL, gU = self._gaps(y)
        if np.any(gL[self.hasL] <= 0) or np.any(gU[self.hasU] <= 0) or (nlp.m_d and np.any(s <= 0)):
            return np.inf
        v = nlp.f(y) - mu * np.sum(np.log(gL[self.hasL])) - mu * np.sum(np.log(gU[self.hasU]))
        viol = np.sum(np.abs(nlp.cons_c(y)))
        if nlp.m_d:
            v -= mu * np.sum(np.log(s))
            viol += np.sum(np.abs(nlp.cons_d(y) + s))
        return v + pen * viol

    def solve(self, y0) -> RefResult:
        nlp = self.nlp
        n, mc, md = nlp.n, nlp.m_c, nlp.m_d
        lb, ub = nlp.lb, nlp.ub
        mu = self.mu0
        # start inside the bounds (1e-2 of the magnitude / range, as the lifted method's cold start)
        y = np.array(y0, dtype=np.float64)
        both = self.hasL & self.hasU
        pl = np.where(self.hasL, 1e-2 * np.maximum(1.0, np.abs(lb)), 0.0)
        pu = np.where(self.hasU, 1e-2 * np.maximum(1.0, np.abs(ub)), 0.0)
        pl = np.where(both, np.minimum(pl, 0.5e-2 * (ub - lb)), pl)
        pu = np.where(both, np.minimum(pu, 0.5e-2 * (ub - lb)), pu)
        y = np.where(self.hasL, np.maximum(y, lb + pl), y)
        y = np.where(self.hasU, np.minimum(y, ub - pu), y)
        s = np.maximum(-nlp.cons_d(y), 1e-2) if md else np.zeros(0)
        lam, nu = np.zeros(mc), mu / s if md else np.zeros(0)
        zs = nu.copy()
        gL, gU = self._gaps(y)
        zL, zU = np.where(self.hasL, mu / gL, 0.0), np.where(self.hasU, mu / gU, 0.0)
        pen, dw_last, status, it = 1.0, 0.0, 1, 0
        E0 = np.inf
        while it < self.max_iter:
            E0 = self._errors(y, s, lam, nu, zs, zL, zU, 0.0)
            if E0 <= self.tol:
                status = 0
                break
            while self._errors(y, s, lam, nu, zs, zL, zU, mu) <= 10.0 * mu and mu > self.mu_min:
                mu = max(self.mu_min, min(0.2 * mu, mu ** 1.5))
            tau = max(0.99, 1.0 - mu)
            gL, gU = self._gaps(y)
            Jc, Jd = nlp.jac_c(y).toarray(), (nlp.jac_d(y).toarray() if md else np.zeros((0, n)))
            W = nlp.hess(y, lam, nu).toarray()
            W = np.tril(W) + np.tril(W, -1).T
            sig = np.where(self.hasL, zL / gL, 0.0) + np.where(self.hasU, zU / gU, 0.0)
            ry = (nlp.grad(y) + Jc.T @ lam + (Jd.T @ nu if md else 0.0)
                  - np.where(self.hasL, mu / gL, 0.0) + np.where(self.hasU, mu / gU, 0.0))
            sig_s = zs / s if md else np.zeros(0)
            rhs = np.concatenate([-ry, -nlp.cons_c(y)]
                                 + ([-(nlp.cons_d(y) + s) - (mu / s - nu) / sig_s] if md else []))
            dw, dc = 0.0, 0.0
            while True:
                A = np.zeros((n + mc + md, n + mc + md))
                A[:n, :n] = W + np.diag(sig) + dw * np.eye(n)
                A[n:n + mc, :n] = Jc
                A[:n, n:n + mc] = Jc.T
                A[n:n + mc, n:n + mc] = -dc * np.eye(mc)
                if md:
                    A[n + mc:, :n] = Jd
                    A[:n, n + mc:] = Jd.T
                    A[n + mc:, n + mc:] = -np.diag(1.0 / sig_s)
                Lf, D, perm = sla.ldl(A, lower=True)
                pos, neg, zero = _inertia(D)
                if pos == n and neg == mc + md and zero == 0:
                    break
                if zero > 0 and dc == 0.0:
                    dc = 1e-8 * mu ** 0.25
                dw = (1e-4 if dw_last == 0.0 else max(1e-20, dw_last / 3.0)) if dw == 0.0 else dw * (100.0 if dw_last == 0.0 else 8.0)
                if dw > 1e40:
                    return RefResult(3, it, y, lam, nu, zL, zU, E0, mu)
            if dw > 0.0:
                dw_last = dw
            sol = sla.solve(A, rhs, assume_a="sym")
            dy, dlam, dnu = sol[:n], sol[n:n + mc], sol[n + mc:]
            ds = (mu / s - nu - dnu) / sig_s if md else np.zeros(0)
            dzs = mu / s - zs - sig_s * ds if md else np.zeros(0)
            dzL = np.where(self.hasL, mu / gL - zL - (zL / gL) * dy, 0.0)
            dzU = np.where(self.hasU, mu / gU - zU + (zU / gU) * dy, 0.0)
            ap = 1.0
            if np.any(self.hasL):
                ap = min(ap, _ftb(gL[self.hasL], dy[self.hasL], tau))
            if np.any(self.hasU):
                ap = min(ap, _ftb(gU[self.hasU], -dy[self.hasU], tau))
            if md:
                ap = min(ap, _ftb(s, ds, tau))
            ad = 1.0
            if md:
                ad = min(ad, _ftb(zs, dzs, tau))
            if np.any(self.hasL):
                ad = min(ad, _ftb(zL[self.hasL], dzL[self.hasL], tau))
            if np.any(self.hasU):
                ad = min(ad, _ftb(zU[self.hasU], dzU[self.hasU], tau))
            pen = max(pen, float(np.max(np.abs(np.concatenate([lam + dlam, nu + dnu, [0.0]])))) + 1.0)
            phi0 = self._phi(y, s, mu, pen)
            viol = np.sum(np.abs(nlp.cons_c(y))) + (np.sum(np.abs(nlp.cons_d(y) + s)) if md else 0.0)
            dphi = (float(nlp.grad(y) @ dy) - mu * float(np.sum(np.where(self.hasL, dy / gL, 0.0)))
                    + mu * float(np.sum(np.where(self.hasU, dy / gU, 0.0))) - pen * viol)
            if md:
                dphi -= mu * float(np.sum(ds / s))
            alpha, ok = ap, False
            for _ in range(60):
                if self._phi(y + alpha * dy, s + alpha * ds, mu, pen) <= phi0 + 1e-4 * alpha * dphi + 1e-14 * abs(phi0):
                    ok = True
                    break
                alpha *= 0.5
            if not ok:
                return RefResult(2, it, y, lam, nu, zL, zU, E0, mu)
            y, s = y + alpha * dy, s + alpha * ds
            lam, nu = lam + alpha * dlam, nu + alpha * dnu
            zs, zL, zU = zs + ad * dzs, zL + ad * dzL, zU + ad * dzU
            # keep the bound multipliers within 1e10 of their primal estimate
            gL, gU = self._gaps(y)
            zL = np.where(self.hasL, np.clip(zL, mu / (1e10 * gL), 1e10 * mu / gL), 0.0)
            zU = np.where(self.hasU, np.clip(zU, mu / (1e10 * gU), 1e10 * mu / gU), 0.0)
            if md:
                zs = np.clip(zs, mu / (1e10 * s), 1e10 * mu / s)
            it += 1
        return RefResult(status, it, y, lam, nu, zL, zU, E0, mu)
