"""Host evaluation of the stage-pattern front end's expressions (test
infrastructure): walks the expression trees of a derived model with NumPy
scalars and expands the per-stage values over a horizon, in the order the
library's pattern uses, so they can be compared with the oracle's own
functions.  Nothing here runs in a solve."""
from __future__ import annotations

import math

import numpy as np

_FN = {"sin": math.sin, "cos": math.cos, "exp": math.exp, "log": math.log, "sqrt": math.sqrt}


def ev(e, env, memo=None):
    memo = {} if memo is None else memo
    got = memo.get(e)
    if got is not None:
        return got
    op = e.op
    if op == "c":
        v = e.args[0]
    elif op == "s":
        v = env[(e.args[0], e.args[1])]
    elif op == "+":
        v = ev(e.args[0], env, memo) + ev(e.args[1], env, memo)
    elif op == "neg":
        v = -ev(e.args[0], env, memo)
    elif op == "*":
        v = ev(e.args[0], env, memo) * ev(e.args[1], env, memo)
    elif op == "pow":
        v = ev(e.args[0], env, memo) ** e.args[1]
    else:
        v = _FN[op](ev(e.args[0], env, memo))
    memo[e] = v
    return v


def stage_env(d, y, k, x0, dt, setpoint=(), traj=None, lam=None, extra=None):
    """Symbol values of stage k (0-based)."""
    m = d.model
    ns = m.ns
    V = y[k * ns:(k + 1) * ns]
    P = y[(k - 1) * ns:(k - 1) * ns + m.nx] if k > 0 else x0
    env = {("dt", 0): dt, ("tr", 0): 0.0 if traj is None else traj[k]}
    for j in range(m.nx):
        env[("x", j)] = V[j]
        env[("px", j)] = P[j]
    for j in range(m.nu):
        env[("u", j)] = V[m.nx + j]
    for j in range(len(m.algebraic)):
        env[("a", j)] = V[m.nx + m.nu + j]
    for j, v in enumerate(setpoint):
        env[("sp", j)] = v
    if lam is not None:
        for r in range(m.rps):
            env[("l", r)] = lam[k * m.rps + r]
    if extra:
        env.update(extra)
    return env


def expand(d, y, H, x0, dt, setpoint=(), traj=None, lam=None):
    """f, grad, c, Jacobian values in the library's row order (previous-stage
    columns first for stages after the first), Hessian values per stage slot,
    with the (row, col) of each entry."""
    m = d.model
    ns, rps = m.ns, m.rps
    f = 0.0
    grad = np.zeros(H * ns)
    c = np.zeros(H * rps)
    jv, jr, jc, wv, wr, wc = [], [], [], [], [], []
    for k in range(H):
        env = stage_env(d, y, k, x0, dt, setpoint, traj, lam)
        memo = {}
        f += ev(m.objective, env, memo)
        for j in range(ns):
            grad[k * ns + j] = ev(d.grad[j], env, memo)
        for r in range(rps):
            c[k * rps + r] = ev(d.rows[r], env, memo)
            if k > 0:
                for col, coef in zip(d.pcols[r], d.pcoef[r]):
                    jv.append(coef)
                    jr.append(k * rps + r)
                    jc.append((k - 1) * ns + col)
            for col, e in zip(d.jcols[r], d.jexpr[r]):
                jv.append(ev(e, env, memo))
                jr.append(k * rps + r)
                jc.append(k * ns + col)
        if lam is not None:
            for (a, b), e in zip(d.wslots, d.wexpr):
                wv.append(ev(e, env, memo))
                wr.append(k * ns + a)
                wc.append(k * ns + b)
    return dict(f=f, grad=grad, c=c, jv=np.array(jv), jr=np.array(jr), jc=np.array(jc), wv=np.array(wv),
                wr=np.array(wr), wc=np.array(wc))


def contraction(d, y, H, x0, dt, setpoint, traj, lam, al, w, so):
    """The parameter contractions the adjoint kernel computes: per setpoint
    entry (summed over stages) and per stage for the trajectory."""
    m = d.model
    ns, rps = m.ns, m.rps
    gsp = np.zeros(m.n_setpoint)
    gtr = np.zeros(H)
    for k in range(H):
        extra = {("so", 0): so}
        for r in range(rps):
            extra[("al", r)] = al[k * rps + r]
        for j in range(ns):
            extra[("w", j)] = w[k * ns + j]
        env = stage_env(d, y, k, x0, dt, setpoint, traj, lam, extra)
        memo = {}
        for j in range(m.n_setpoint):
            gsp[j] += ev(d.adj_sp[j], env, memo)
        gtr[k] = ev(d.adj_tr, env, memo)
    return gsp, gtr
