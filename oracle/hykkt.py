"""HyKKT interior-point method (oracle side; test infrastructure only, never
imported by the library).

Section 3.2 names two ways to make the condensed system of eq. (14) solvable
by a Cholesky factorization: Lifted-KKT (eq. 16, ``oracle/ipm.py``) and HyKKT,
the hybrid direct-iterative method of the augmented-Lagrangian literature the
paper cites.  HyKKT keeps the equalities exact.  The condensed system of
eq. (14),

    [ K_c  H^T ] [dy     ]   [ b1 ]      K_c = W + Sigma + eta I + J_d^T Q_d J_d
    [ H    0   ] [dlambda] = [ b2 ]      H = J_c,  b1 = -r1 - J_d^T (Q_d r4_d - r2_d),  b2 = -c

is rewritten with gamma_h > 0 (the first block row plus gamma_h H^T times the
second) as

    K_gamma dy + H^T dlambda = b1 + gamma_h H^T b2,     K_gamma = K_c + gamma_h H^T H,

so that, with the Cholesky factor of K_gamma (positive definite when K_c is
positive definite on the null space of H and gamma_h is large enough), the
multiplier step solves the Schur-complement system

    S dlambda = H K_gamma^{-1} (b1 + gamma_h H^T b2) - b2,    S = H K_gamma^{-1} H^T

by conjugate gradients (S is symmetric positive definite; each product with S
is one forward/back solve with the factor), and then
dy = K_gamma^{-1} (b1 + gamma_h H^T b2 - H^T dlambda).  A failed factorization
raises eta as in the inertia correction of eqs. (12)-(13); K_gamma has the
sparsity pattern of the lifted matrix, so the symbolic analysis is the same.

The rest of the method is Algorithm 2 as the lifted oracle runs it (filter
line search and the l1-merit fallback, barrier update, termination, one step
length for the whole iterate; no second-order corrections, each of which would
need a conjugate-gradient solve of its own), applied to the
problem without the lifting: min f(y) s.t. c(y) = 0, d(y) + s = 0, s >= 0,
lb <= y <= ub.  The state reuses the lifted one with these meanings:
s holds the slacks of the m_d inequality rows, omega = [lambda; nu] (equality
multipliers, free; inequality multipliers), beta the duals of s, and the
constraint residual is r4 = [c; d + s], so theta = |c|_1 + |d + s|_1.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .ipm import IPMOptions, IPMState, LiftedIPM


@dataclass
class HyKKTOptions:
    gamma_h: float = 1e6       # weight of H^T H in K_gamma
    cg_tol: float = 1e-12      # CG stops at |r|_2 <= cg_tol |b|_2
    cg_max: int = 200          # CG iterations per solve


def hykkt_solve(chol, H, b1, b2, gamma_h, cg_tol, cg_max):
    """The 2 x 2 condensed system by HyKKT; ``chol`` holds the Cholesky factor
    of K_gamma.  Returns (dy, dlambda, CG iterations, converged)."""
    rhs = b1 + gamma_h * (H.T @ b2)
    w0 = chol.solve(rhs)
    bS = H @ w0 - b2
    x = np.zeros(H.shape[0])
    r = bS.copy()
    p = r.copy()
    rr = float(r @ r)
    stop = cg_tol * np.sqrt(rr)
    it, ok = 0, rr == 0.0
    while not ok and it < cg_max:
        Sp = H @ chol.solve(H.T @ p)
        a = rr / float(p @ Sp)
        x += a * p
        r -= a * Sp
        rr_new = float(r @ r)
        it += 1
        if np.sqrt(rr_new) <= stop:
            ok = True
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    dy = chol.solve(rhs - H.T @ x)
    return dy, x, it, ok


class HyKKTIPM(LiftedIPM):
    def __init__(self, nlp, opts: IPMOptions | None = None, hopts: HyKKTOptions | None = None):
        # no second-order corrections: each would need its own CG solve
        super().__init__(nlp, dataclasses.replace(opts or IPMOptions(), soc_max=0))
        self.h = hopts or HyKKTOptions()
        self.ml = self.mc + self.md      # rows of omega: [c rows; d rows]
        self.cg_total = 0

    # ---- state ----------------------------------------------------------------
    def cold_start(self, y_guess, mu0):
        """y pushed inside its bounds as in the lifted cold start; inequality
        slacks s = max(-d, slack_push max(1, |d|)); omega = 0; beta = mu0 / s;
        zL, zU = mu0 / gaps."""
        st = super().cold_start(y_guess, mu0)      # y and the bound duals
        d = self.nlp.cons_d(st.y)
        s = np.maximum(-d, self.o.slack_push * np.maximum(1.0, np.abs(d)))
        return IPMState(st.y, s, np.zeros(self.ml), mu0 / s, st.zL, st.zU)

    def from_lifted(self, st):
        """A Lifted-KKT iterate as a HyKKT one: lambda = omega+ - omega-; the
        inequality rows' slack, multiplier and dual kept."""
        mc = self.mc
        om = np.concatenate([st.omega[:mc] - st.omega[mc:2 * mc], st.omega[2 * mc:]])
        return IPMState(st.y.copy(), st.s[2 * mc:].copy(), om, st.beta[2 * mc:].copy(), st.zL.copy(),
                        st.zU.copy())

    def multipliers(self, st):
        return st.omega[:self.mc], st.omega[self.mc:]

    # ---- residuals ----------------------------------------------------------
    def constraint_residual(self, y, s):
        """r4 = [c(y); d(y) + s]."""
        return np.concatenate([self.nlp.cons_c(y), self.nlp.cons_d(y) + s])

    def _dual(self, st, gf, Jc, Jd):
        lam, nu = self.multipliers(st)
        out = gf + Jc.T @ lam
        if self.md:
            out = out + Jd.T @ nu
        return out

    def errors(self, st, gf, c, d, Jc, Jd, mu):
        gL, gU = self.gaps(st.y)
        dual = self._dual(st, gf, Jc, Jd) - st.zL + st.zU
        e = [np.max(np.abs(dual))]
        if self.mc:
            e.append(np.max(np.abs(c)))
        if self.md:
            nu = st.omega[self.mc:]
            e += [np.max(np.abs(nu - st.beta)), np.max(np.abs(d + st.s)), np.max(np.abs(st.s * st.beta - mu))]
        if np.any(self.hasL):
            e.append(np.max(np.abs((gL * st.zL - mu)[self.hasL])))
        if np.any(self.hasU):
            e.append(np.max(np.abs((gU * st.zU - mu)[self.hasU])))
        return float(max(e))

    # ---- the Newton direction by HyKKT --------------------------------------
    def newton_step(self, st, mu, f, gf, c, d, Jc, Jd):
        o, h, nlp, mc = self.o, self.h, self.nlp, self.mc
        lam, nu = self.multipliers(st)
        W = nlp.hess(st.y, lam, nu)
        gL, gU = self.gaps(st.y)
        sigL = np.where(self.hasL, st.zL / gL, 0.0)
        sigU = np.where(self.hasU, st.zU / gU, 0.0)
        r1 = (self._dual(st, gf, Jc, Jd) - np.where(self.hasL, mu / gL, 0.0)
              + np.where(self.hasU, mu / gU, 0.0))
        Kc = W + sp.diags(sigL + sigU)
        if self.md:
            Q = st.beta / st.s
            r2 = nu - mu / st.s
            Kc = Kc + Jd.T @ sp.diags(Q) @ Jd
        else:
            Q = r2 = np.zeros(0)
        Kg = (Kc + h.gamma_h * (Jc.T @ Jc)).tocsr()
        eta = 0.0
        ok = self.chol.factor(Kg)
        if not ok:
            eta = o.eta_first if self.eta_last == 0.0 else max(o.eta_min, o.km * self.eta_last)
            while True:
                ok = self.chol.factor(Kg + eta * sp.identity(self.n, format="csr"))
                if ok:
                    break
                eta *= o.kp_first if self.eta_last == 0.0 else o.kp
                if eta > o.eta_max:
                    return None
            self.eta_last = eta
        self._soc_ctx = (r1, r2, Q, Jc, Jd, gL, gU, sigL, sigU, mu, st)
        r4 = np.concatenate([c, d + st.s])
        out = self._directions(r4)
        out.update(eta=eta, r4=r4, K=(Kc + eta * sp.identity(self.n)).tocsr(), Kg=Kg)
        return out

    def _directions(self, r4):
        """Directions of the last Newton system (same factor) for the
        constraint residual r4 = [r4_c; r4_d]."""
        h, mc = self.h, self.mc
        r1, r2, Q, Jc, Jd, gL, gU, sigL, sigU, mu, st = self._soc_ctx
        b1 = -r1
        if self.md:
            b1 = b1 - Jd.T @ (Q * r4[mc:] - r2)
        dy, dlam, it, ok = hykkt_solve(self.chol, Jc, b1, -r4[:mc], h.gamma_h, h.cg_tol, h.cg_max)
        self.cg_total += it
        if self.md:
            ds = -r4[mc:] - Jd @ dy
            dnu = -r2 - Q * ds
            dbe = mu / st.s - st.beta - Q * ds
        else:
            ds = dnu = dbe = np.zeros(0)
        dzL = np.where(self.hasL, mu / gL - st.zL - sigL * dy, 0.0)
        dzU = np.where(self.hasU, mu / gU - st.zU + sigU * dy, 0.0)
        return dict(dy=dy, ds=ds, domega=np.concatenate([dlam, dnu]), dbeta=dbe, dzL=dzL, dzU=dzU,
                    cg_iters=it, cg_ok=ok)

    def soc_direction(self, r4s):
        d = self._directions(r4s)
        return d["dy"], d["ds"], d["domega"], d["dbeta"], d["dzL"], d["dzU"]
