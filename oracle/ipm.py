"""Lifted-KKT primal-dual interior-point method (oracle side), Section 3.2,
Algorithm 2.

Problem (eq. 6, with variable bounds kept as barrier terms as the -mu Y^{-1} e
term of r_1 in eq. 11 implies):
    min f(y)  s.t.  c(y) = 0,  d(y) <= 0,  lb <= y <= ub.
Lifting (eq. 16): the equalities are relaxed to -gamma <= c <= gamma, so the
inequality rows become  g^l = [c - gamma; -c - gamma; d]  (m^l = 2 m_c + m_d),
with slacks s >= 0, g^l + s = 0, multipliers omega (for g^l + s = 0), beta
(for s >= 0), zL / zU (for the bounds).

One Newton iteration (eqs. 10-11, 14, 17, 22-25):
    r1 = grad f + G^T omega - mu/(y - lb) + mu/(ub - y)
    r2 = omega - mu / s
    r4 = g^l + s
    Q  = beta / s,   Sigma = zL/(y - lb) + zU/(ub - y)
    K  = W + Sigma + eta I + G^T Q G        (W = Hessian of f + lam^T c, lam = omega+ - omega-)
    K dy = -r1 - G^T (Q r4 - r2)            (solved by Cholesky; failure -> larger eta)
    ds = -r4 - G dy;   domega = -r2 - Q ds
    dbeta = mu/s - beta - Q ds
    dzL = mu/(y-lb) - zL - Sigma_L dy,  dzU = mu/(ub-y) - zU + Sigma_U dy
Step (eq. 26): one alpha for the whole primal-dual vector z, from a
backtracking line search started at the fraction-to-boundary limit of every
positive quantity (s, bound gaps, beta, zL, zU).  A single step keeps
omega - beta shrinking by (1 - alpha) per iteration; the lifted multipliers
grow like mu / gamma away from the solution, so separate primal and dual steps
would let that difference blow up.  The line search is the filter method of
the interior-point reference the paper builds on (Waechter and Biegler): a
trial point is judged by the constraint violation theta = |g^l + s|_1 and the
barrier objective phi = f - mu (sum ln s + sum ln bound gaps) against a filter
of (theta, phi) pairs that is reset whenever mu changes; an Armijo decrease of
phi is required when theta is small and the step is a descent direction (the
switching condition), sufficient decrease of theta or phi otherwise.  When
the first trial point is rejected and does not reduce theta, up to soc_max
second-order corrections are tried: the step is recomputed with the same
factor from the residual alpha r4 + (g^l + s) at the trial point (accumulated
over corrections) and taken, with its own fraction-to-boundary step, if the
filter accepts it.  No restoration phase: a step below the minimal step length
ends the solve with status 2.  Barrier update after the inner test
(eq. 27), termination on the mu = 0 optimality error (eq. 28).

The constants the paper leaves open are fixed in ``IPMOptions``; the GPU library
uses the same values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

EPS = np.finfo(np.float64).eps


@dataclass
class IPMOptions:
    tol: float = 1e-8            # epsilon_outer on E_0
    gamma: float = 1e-9          # equality relaxation of the lifting
    mu0_cold: float = 1e-1
    mu0_warm: float = 1e-9       # warm start at the final barrier value
    mu_min: float = 1e-9
    kappa_eps: float = 10.0      # inner test: E_mu <= kappa_eps * mu
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    armijo: float = 1e-4
    ls_max: int = 40
    kappa_sigma: float = 1e10
    max_iter: int = 200
    eta_first: float = 1e-4
    eta_min: float = 1e-20
    eta_max: float = 1e40
    kp_first: float = 100.0
    kp: float = 8.0
    km: float = 1.0 / 3.0
    bound_push: float = 1e-2
    slack_push: float = 1e-2
    # filter line search
    filter_gamma_theta: float = 1e-5
    filter_gamma_phi: float = 1e-8
    filter_s_theta: float = 1.1
    filter_s_phi: float = 2.3
    filter_delta: float = 1.0
    alpha_min_frac: float = 0.05
    theta_max_fact: float = 1e4
    theta_min_fact: float = 1e-4
    filter_cap: int = 128
    soc_max: int = 4            # second-order corrections per line search
    soc_kappa: float = 0.99     # each correction must reduce theta by this factor
    merit_fallback: int = 1     # l1-merit backtracking when the filter rejects every trial


STATUS = {0: "converged", 1: "max_iter", 2: "linesearch_fail", 3: "regularization_fail",
          4: "nonfinite"}


@dataclass
class IPMState:
    y: np.ndarray
    s: np.ndarray
    omega: np.ndarray
    beta: np.ndarray
    zL: np.ndarray
    zU: np.ndarray

    def copy(self):
        return IPMState(*(a.copy() for a in (self.y, self.s, self.omega, self.beta, self.zL, self.zU)))


@dataclass
class IPMResult:
    status: int
    iters: int
    state: IPMState
    mu: float
    eta: float
    E0: float
    trace: list = field(default_factory=list)


def _ftb(v, dv, tau):
    """Largest alpha in (0, 1] with v + alpha dv >= (1 - tau) v (v > 0)."""
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))


class CholeskySolver:
    """Cholesky of an SPD matrix given in CSR; banded storage when the natural
    order has a narrow band, dense otherwise.  ``factor`` returns False when the
    matrix is not numerically positive definite (a pivot <= 0 or non-finite)."""

    def __init__(self, n, pattern_rows, pattern_cols):
        self.n = n
        bw = int(np.max(np.abs(np.asarray(pattern_rows) - np.asarray(pattern_cols)))) if len(pattern_rows) else 0
        self.bw = bw
        self.banded = (bw + 1) * 4 < n

    def factor(self, K):
        K = K.tocsr()
        if not np.all(np.isfinite(K.data)):
            return False
        try:
            if self.banded:
                Kc = K.tocoo()
                ab = np.zeros((self.bw + 1, self.n))
                low = Kc.row >= Kc.col
                ab[(Kc.row - Kc.col)[low], Kc.col[low]] = Kc.data[low]
                self.cb = sla.cholesky_banded(ab, lower=True)
            else:
                self.L = np.linalg.cholesky(K.toarray())
        except (np.linalg.LinAlgError, sla.LinAlgError):
            return False
        return True

    def solve(self, b):
        if self.banded:
            return sla.cho_solve_banded((self.cb, True), b)
        return sla.cho_solve((self.L, True), b)


class LiftedIPM:
    def __init__(self, nlp, opts: IPMOptions | None = None):
        self.nlp = nlp
        self.o = opts or IPMOptions()
        self.n, self.mc, self.md = nlp.n, nlp.m_c, nlp.m_d
        self.ml = 2 * self.mc + self.md
        self.hasL = np.isfinite(nlp.lb)
        self.hasU = np.isfinite(nlp.ub)
        from .symbolic import kkt_lower_pattern
        r, c = kkt_lower_pattern(nlp)
        self.chol = CholeskySolver(self.n, r, c)
        self.eta_last = 0.0

    # ---- lifted constraint helpers ----------------------------------
    def g_lifted(self, c, d):
        g = self.o.gamma
        return np.concatenate([c - g, -c - g, d])

    def GT(self, Jc, Jd, v):
        mc = self.mc
        out = Jc.T @ (v[:mc] - v[mc:2 * mc])
        if self.md:
            out = out + Jd.T @ v[2 * mc:]
        return out

    def G(self, Jc, Jd, dy):
        a = Jc @ dy
        parts = [a, -a]
        if self.md:
            parts.append(Jd @ dy)
        return np.concatenate(parts)

    def gaps(self, y):
        gl = np.where(self.hasL, y - self.nlp.lb, 1.0)
        gu = np.where(self.hasU, self.nlp.ub - y, 1.0)
        return gl, gu

    # ---- starting points ---------------------------------------------
    def cold_start(self, y_guess, mu0):
        o, nlp = self.o, self.nlp
        lb, ub = nlp.lb, nlp.ub
        y = np.array(y_guess, dtype=np.float64)
        # push into the interior (fraction of the bound magnitude and of the range)
        pl = np.where(self.hasL, o.bound_push * np.maximum(1.0, np.abs(lb)), 0.0)
        pu = np.where(self.hasU, o.bound_push * np.maximum(1.0, np.abs(ub)), 0.0)
        both = self.hasL & self.hasU
        rng = np.where(both, ub - lb, np.inf)
        pl = np.where(both, np.minimum(pl, 0.5 * o.bound_push * rng), pl)
        pu = np.where(both, np.minimum(pu, 0.5 * o.bound_push * rng), pu)
        y = np.where(self.hasL, np.maximum(y, lb + pl), y)
        y = np.where(self.hasU, np.minimum(y, ub - pu), y)
        gl = self.g_lifted(nlp.cons_c(y), nlp.cons_d(y))
        s = np.maximum(-gl, o.slack_push * np.maximum(1.0, np.abs(gl)))
        omega = np.zeros(self.ml)
        beta = mu0 / s
        gL, gU = self.gaps(y)
        zL = np.where(self.hasL, mu0 / gL, 0.0)
        zU = np.where(self.hasU, mu0 / gU, 0.0)
        return IPMState(y, s, omega, beta, zL, zU)

    # ---- optimality errors -------------------------------------------
    def errors(self, st, gf, c, d, Jc, Jd, mu):
        gL, gU = self.gaps(st.y)
        dual = gf + self.GT(Jc, Jd, st.omega) - st.zL + st.zU
        prim = self.g_lifted(c, d) + st.s
        e = [np.max(np.abs(dual)), np.max(np.abs(st.omega - st.beta)), np.max(np.abs(prim)),
             np.max(np.abs(st.s * st.beta - mu))]
        if np.any(self.hasL):
            e.append(np.max(np.abs((gL * st.zL - mu)[self.hasL])))
        if np.any(self.hasU):
            e.append(np.max(np.abs((gU * st.zU - mu)[self.hasU])))
        return float(max(e))

    def barrier_objective(self, y, s, mu, fval):
        """phi_mu = f - mu sum ln s - mu sum ln(bound gaps)."""
        gL, gU = self.gaps(y)
        phi = fval - mu * np.sum(np.log(s))
        if np.any(self.hasL):
            phi -= mu * np.sum(np.log(gL[self.hasL]))
        if np.any(self.hasU):
            phi -= mu * np.sum(np.log(gU[self.hasU]))
        return float(phi)

    def constraint_residual(self, y, s):
        """g^l(y) + s (r_4 of eq. 11 at y, s)."""
        return self.g_lifted(self.nlp.cons_c(y), self.nlp.cons_d(y)) + s

    def violation(self, y, s):
        """theta = |g^l(y) + s|_1."""
        return float(np.sum(np.abs(self.constraint_residual(y, s))))

    # ---- main loop ----------------------------------------------------
    def solve(self, start: IPMState, mu0: float, record=False, fixed_mu=False, tol=None, progress=None):
        """Algorithm 2 from ``start`` with initial barrier value mu0.  With
        ``fixed_mu`` the barrier value is never decreased and the loop stops when
        E_mu <= tol (Newton's method on one barrier problem, used for finite
        differences of the barrier solution).  ``progress(it, mu, E0)``, when
        given, is called once per iteration (logging only)."""
        o, nlp = self.o, self.nlp
        tol = o.tol if tol is None else tol
        st = start.copy()
        mu = mu0
        self.eta_last = 0.0
        theta_max = theta_min = None
        filt = []            # (theta, phi) pairs, insertion order
        filt_mu = None
        nu = 1.0
        trace = []
        status = 1
        it = 0
        eta = 0.0
        E0 = np.inf
        while True:
            f = nlp.f(st.y)
            gf = nlp.grad(st.y)
            c, d = nlp.cons_c(st.y), nlp.cons_d(st.y)
            Jc, Jd = nlp.jac_c(st.y), nlp.jac_d(st.y)
            if not (np.isfinite(f) and np.all(np.isfinite(gf)) and np.all(np.isfinite(c))):
                status = 4
                break
            E0 = self.errors(st, gf, c, d, Jc, Jd, 0.0)
            if progress is not None:
                progress(it, mu, E0)
            if fixed_mu:
                if self.errors(st, gf, c, d, Jc, Jd, mu) <= tol:
                    status = 0
                    break
            elif E0 <= tol:
                status = 0
                break
            if it >= o.max_iter:
                status = 1
                break
            # barrier update (eq. 27 inner test, Algorithm 2 outer loop)
            Emu = self.errors(st, gf, c, d, Jc, Jd, mu)
            while not fixed_mu and Emu <= o.kappa_eps * mu and mu > o.mu_min:
                mu = max(o.mu_min, min(o.kappa_mu * mu, mu ** o.theta_mu))
                Emu = self.errors(st, gf, c, d, Jc, Jd, mu)
            tau = max(o.tau_min, 1.0 - mu)
            step = self.newton_step(st, mu, f, gf, c, d, Jc, Jd)
            if step is None:
                status = 3
                break
            eta = step["eta"]
            dy, ds, dom, dbe, dzL, dzU = (step[k] for k in ("dy", "ds", "domega", "dbeta", "dzL", "dzU"))
            r4 = step["r4"]
            gL, gU = self.gaps(st.y)
            # fraction to boundary
            amax = _ftb(st.s, ds, tau)
            if np.any(self.hasL):
                amax = min(amax, _ftb(gL[self.hasL], dy[self.hasL], tau))
            if np.any(self.hasU):
                amax = min(amax, _ftb(gU[self.hasU], -dy[self.hasU], tau))
            adu = _ftb(st.beta, dbe, tau)
            if np.any(self.hasL):
                adu = min(adu, _ftb(st.zL[self.hasL], dzL[self.hasL], tau))
            if np.any(self.hasU):
                adu = min(adu, _ftb(st.zU[self.hasU], dzU[self.hasU], tau))
            # filter line search (eq. 26)
            theta = float(np.sum(np.abs(r4)))
            phi0 = self.barrier_objective(st.y, st.s, mu, f)
            Dphi = (float(gf @ dy) - mu * float(np.sum(ds / st.s))
                    - mu * float(np.sum(np.where(self.hasL, dy / gL, 0.0)))
                    + mu * float(np.sum(np.where(self.hasU, dy / gU, 0.0))))
            if it == 0:
                theta_max = o.theta_max_fact * max(1.0, theta)
                theta_min = o.theta_min_fact * max(1.0, theta)
            if mu != filt_mu:
                filt = []
                filt_mu = mu
            g_th, g_ph, s_th, s_ph, dl = (o.filter_gamma_theta, o.filter_gamma_phi, o.filter_s_theta,
                                          o.filter_s_phi, o.filter_delta)
            if Dphi < 0.0:
                amin = min(g_th, g_ph * theta / (-Dphi))
                if theta <= theta_min:
                    amin = min(amin, dl * theta ** s_th / (-Dphi) ** s_ph)
            else:
                amin = g_th
            amin *= o.alpha_min_frac
            alpha = min(amax, adu)
            accepted = False
            trials = 0
            soc_dir = None

            def acceptable(tht, pht, a):
                nonlocal filt
                ok = np.isfinite(tht) and np.isfinite(pht) and tht < theta_max
                if ok:
                    ok = all(tht < tf or pht < pf for (tf, pf) in filt)
                if not ok:
                    return False
                switching = (Dphi < 0.0 and theta <= theta_min and a * (-Dphi) ** s_ph > dl * theta ** s_th)
                if switching:
                    return pht <= phi0 + o.armijo * a * Dphi + 10.0 * EPS * abs(phi0)
                acc = tht <= (1.0 - g_th) * theta or pht <= phi0 - g_ph * theta
                if acc:
                    entry = ((1.0 - g_th) * theta, phi0 - g_ph * theta)
                    filt = [e for e in filt if not (e[0] >= entry[0] and e[1] >= entry[1])]
                    if len(filt) >= o.filter_cap:
                        filt.pop(0)
                    filt.append(entry)
                return acc

            while alpha >= amin and trials < o.ls_max:
                trials += 1
                yt = st.y + alpha * dy
                stt = st.s + alpha * ds
                tht = self.violation(yt, stt)
                pht = self.barrier_objective(yt, stt, mu, nlp.f(yt))
                if acceptable(tht, pht, alpha):
                    accepted = True
                    break
                if trials == 1 and np.isfinite(tht) and tht >= theta and o.soc_max > 0:
                    r4s = alpha * r4 + self.constraint_residual(yt, stt)
                    th_old = theta
                    for _p in range(o.soc_max):
                        d = self.soc_direction(r4s)
                        a_s = _ftb(st.s, d[1], tau)
                        if np.any(self.hasL):
                            a_s = min(a_s, _ftb(gL[self.hasL], d[0][self.hasL], tau))
                        if np.any(self.hasU):
                            a_s = min(a_s, _ftb(gU[self.hasU], -d[0][self.hasU], tau))
                        a_s = min(a_s, _ftb(st.beta, d[3], tau))
                        if np.any(self.hasL):
                            a_s = min(a_s, _ftb(st.zL[self.hasL], d[4][self.hasL], tau))
                        if np.any(self.hasU):
                            a_s = min(a_s, _ftb(st.zU[self.hasU], d[5][self.hasU], tau))
                        ys, ss = st.y + a_s * d[0], st.s + a_s * d[1]
                        ths = self.violation(ys, ss)
                        phs = self.barrier_objective(ys, ss, mu, nlp.f(ys))
                        if acceptable(ths, phs, alpha):
                            soc_dir = d
                            alpha = a_s
                            accepted = True
                            break
                        if not np.isfinite(ths) or ths > o.soc_kappa * th_old:
                            break
                        r4s = a_s * r4s + self.constraint_residual(ys, ss)
                        th_old = ths
                    if accepted:
                        break
                alpha *= 0.5
            merit = False
            if not accepted and o.merit_fallback:
                nu = max(nu, float(np.max(np.abs(st.omega + dom))) + 1.0)
                m0 = phi0 + nu * theta
                Dm = Dphi - nu * theta
                alpha = min(amax, adu)
                for _t in range(o.ls_max):
                    trials += 1
                    yt = st.y + alpha * dy
                    stt = st.s + alpha * ds
                    mt = self.barrier_objective(yt, stt, mu, nlp.f(yt)) + nu * self.violation(yt, stt)
                    if np.isfinite(mt) and mt <= m0 + o.armijo * alpha * Dm + 10.0 * EPS * abs(m0):
                        accepted = merit = True
                        filt = []
                        break
                    alpha *= 0.5
            if soc_dir is not None:
                dy, ds, dom, dbe, dzL, dzU = soc_dir
            if record:
                trace.append(dict(it=it, mu=mu, eta=eta, amax=amax, alpha=alpha, adu=adu,
                                  E0=E0, Emu=Emu, trials=trials, phi=phi0, Dphi=Dphi, theta=theta,
                                  filter=len(filt), merit=merit, dy_norm=float(np.max(np.abs(dy)))))
            if not accepted:
                status = 2
                break
            st.y = st.y + alpha * dy
            st.s = st.s + alpha * ds
            st.omega = st.omega + alpha * dom
            st.beta = st.beta + alpha * dbe
            st.zL = st.zL + alpha * dzL
            st.zU = st.zU + alpha * dzU
            # keep the bound multipliers within kappa_sigma of the primal estimate
            ks = o.kappa_sigma
            st.beta = np.clip(st.beta, mu / (ks * st.s), ks * mu / st.s)
            gL, gU = self.gaps(st.y)
            st.zL = np.where(self.hasL, np.clip(st.zL, mu / (ks * gL), ks * mu / gL), 0.0)
            st.zU = np.where(self.hasU, np.clip(st.zU, mu / (ks * gU), ks * mu / gU), 0.0)
            it += 1
        return IPMResult(status=status, iters=it, state=st, mu=mu, eta=eta, E0=E0, trace=trace)

    def newton_step(self, st, mu, f, gf, c, d, Jc, Jd):
        """Condensed Newton direction at ``st`` (eqs. 10-11, 14, 17, 22-25) with
        inertia correction; returns None when eta exceeds eta_max."""
        o, nlp, mc = self.o, self.nlp, self.mc
        lam = st.omega[:mc] - st.omega[mc:2 * mc]
        lam_d = st.omega[2 * mc:]
        W = nlp.hess(st.y, lam, lam_d)
        gL, gU = self.gaps(st.y)
        sigL = np.where(self.hasL, st.zL / gL, 0.0)
        sigU = np.where(self.hasU, st.zU / gU, 0.0)
        Q = st.beta / st.s
        r1 = (gf + self.GT(Jc, Jd, st.omega)
              - np.where(self.hasL, mu / gL, 0.0) + np.where(self.hasU, mu / gU, 0.0))
        r2 = st.omega - mu / st.s
        r4 = self.g_lifted(c, d) + st.s
        Qc = Q[:mc] + Q[mc:2 * mc]
        JQJ = Jc.T @ sp.diags(Qc) @ Jc
        if self.md:
            JQJ = JQJ + Jd.T @ sp.diags(Q[2 * mc:]) @ Jd
        K0 = (W + sp.diags(sigL + sigU) + JQJ).tocsr()
        rhs = -r1 - self.GT(Jc, Jd, Q * r4 - r2)
        # inertia correction (eqs. 12-13, 15, 17): eta grows until Cholesky succeeds
        eta = 0.0
        ok = self.chol.factor(K0)
        if not ok:
            eta = o.eta_first if self.eta_last == 0.0 else max(o.eta_min, o.km * self.eta_last)
            while True:
                ok = self.chol.factor(K0 + eta * sp.identity(self.n, format="csr"))
                if ok:
                    break
                eta *= o.kp_first if self.eta_last == 0.0 else o.kp
                if eta > o.eta_max:
                    return None
            self.eta_last = eta
        self._soc_ctx = (r1, r2, Q, Jc, Jd, gL, gU, sigL, sigU, mu, st)
        dy = self.chol.solve(rhs)
        ds = -r4 - self.G(Jc, Jd, dy)
        dom = -r2 - Q * ds
        dbe = mu / st.s - st.beta - Q * ds
        dzL = np.where(self.hasL, mu / gL - st.zL - sigL * dy, 0.0)
        dzU = np.where(self.hasU, mu / gU - st.zU + sigU * dy, 0.0)
        return dict(dy=dy, ds=ds, domega=dom, dbeta=dbe, dzL=dzL, dzU=dzU, eta=eta,
                    K=K0, rhs=rhs, W=W, r1=r1, r2=r2, r4=r4, Q=Q, sigL=sigL, sigU=sigU)

    def soc_direction(self, r4s):
        """Directions of the last Newton step's system (same factor) with the
        constraint residual r4 replaced by r4s (a second-order correction)."""
        r1, r2, Q, Jc, Jd, gL, gU, sigL, sigU, mu, st = self._soc_ctx
        rhs = -r1 - self.GT(Jc, Jd, Q * r4s - r2)
        dy = self.chol.solve(rhs)
        ds = -r4s - self.G(Jc, Jd, dy)
        dom = -r2 - Q * ds
        dbe = mu / st.s - st.beta - Q * ds
        dzL = np.where(self.hasL, mu / gL - st.zL - sigL * dy, 0.0)
        dzU = np.where(self.hasU, mu / gU - st.zU + sigU * dy, 0.0)
        return dy, ds, dom, dbe, dzL, dzU

    def multipliers(self, st):
        """Equality multipliers of the original problem: lam = omega+ - omega-."""
        mc = self.mc
        return st.omega[:mc] - st.omega[mc:2 * mc], st.omega[2 * mc:]
