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


def stage_env(d, y, k, x0, dt, setpoint=(), traj=None, lam=None, lam_d=None, u_prev=None, extra=None):
    """Symbol values of stage k (0-based)."""
    m = d.model
    ns = m.ns
    V = y[k * ns:(k + 1) * ns]
    P = y[(k - 1) * ns:(k - 1) * ns + m.nx] if k > 0 else x0
    PU = y[(k - 1) * ns + m.nx:(k - 1) * ns + m.nx + m.nu] if k > 0 else u_prev
    env = {("dt", 0): dt, ("tr", 0): 0.0 if traj is None else traj[k]}
    for j in range(m.nx):
        env[("x", j)] = V[j]
        env[("px", j)] = P[j]
    for j in range(m.nu):
        env[("u", j)] = V[m.nx + j]
        if PU is not None:
            env[("pu", j)] = PU[j]
    for j in range(len(m.algebraic)):
        env[("a", j)] = V[m.nx + m.nu + j]
    for j, v in enumerate(setpoint):
        env[("sp", j)] = v
    if lam is not None:
        for r in range(m.rps):
            env[("l", r)] = lam[k * m.rps + r]
    if lam_d is not None:
        for r in range(m.nd):
            env[("ld", r)] = lam_d[k * m.nd + r]
    if extra:
        env.update(extra)
    return env


def expand(d, y, H, x0, dt, setpoint=(), traj=None, lam=None, lam_d=None, u_prev=None):
    """f, grad, c, d, Jacobian values in the library's row order (equality
    rows with previous-stage columns first for stages after the first, then
    the inequality rows), Hessian values per stage slot (own entries, then
    those with the previous stage's controls), with (row, col) of each."""
    m = d.model
    ns, rps, nd, nx = m.ns, m.rps, m.nd, m.nx
    mc = H * rps
    envs = [stage_env(d, y, k, x0, dt, setpoint, traj, lam, lam_d, u_prev) for k in range(H)]
    memos = [{} for _ in range(H)]
    f = 0.0
    grad = np.zeros(H * ns)
    c = np.zeros(H * rps)
    dv = np.zeros(H * nd)
    jv, jr, jc, wv, wr, wc = [], [], [], [], [], []
    for k in range(H):
        env, memo = envs[k], memos[k]
        nxt = k + 1 < H
        f += ev(m.objective, env, memo)
        for j in range(ns):
            g = ev(d.grad[j], env, memo)
            if nxt:
                g += ev(d.gnext[j], envs[k + 1], memos[k + 1])
            grad[k * ns + j] = g
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
    for k in range(H):
        env, memo = envs[k], memos[k]
        for r in range(nd):
            dv[k * nd + r] = ev(d.drows[r], env, memo)
            for col, e in zip(d.dcols[r], d.dexpr[r]):
                jv.append(ev(e, env, memo))
                jr.append(mc + k * nd + r)
                jc.append(k * ns + col)
    if lam is not None:
        for k in range(H):
            env, memo = envs[k], memos[k]
            for (a, b), e, en in zip(d.wslots, d.wexpr, d.wnext):
                v = ev(e, env, memo)
                if k + 1 < H:
                    v += ev(en, envs[k + 1], memos[k + 1])
                wv.append(v)
                wr.append(k * ns + a)
                wc.append(k * ns + b)
            if k > 0:
                for (a, b), e in zip(d.xslots, d.xexpr):
                    wv.append(ev(e, env, memo))
                    wr.append(k * ns + a)
                    wc.append((k - 1) * ns + nx + b)
    return dict(f=f, grad=grad, c=c, d=dv, jv=np.array(jv), jr=np.array(jr, dtype=int),
                jc=np.array(jc, dtype=int), wv=np.array(wv), wr=np.array(wr, dtype=int),
                wc=np.array(wc, dtype=int))


def contraction(d, y, H, x0, dt, setpoint, traj, lam, al, w, so, lam_d=None, u_prev=None):
    """The parameter contractions the adjoint kernel computes: per setpoint
    entry (summed over stages), per stage for the trajectory, and for the
    last applied control (first stage)."""
    m = d.model
    ns, rps, nd, nx = m.ns, m.rps, m.nd, m.nx
    mc = H * rps
    gsp = np.zeros(m.n_setpoint)
    gtr = np.zeros(H)
    gup = np.zeros(m.nu)
    for k in range(H):
        extra = {("so", 0): so}
        for r in range(rps):
            extra[("al", r)] = al[k * rps + r]
        for r in range(nd):
            extra[("ald", r)] = al[mc + k * nd + r]
        for j in range(ns):
            extra[("w", j)] = w[k * ns + j]
        for b in range(m.nu):
            extra[("wp", b)] = w[(k - 1) * ns + nx + b] if k > 0 else 0.0
        env = stage_env(d, y, k, x0, dt, setpoint, traj, lam, lam_d, u_prev, extra)
        memo = {}
        for j in range(m.n_setpoint):
            gsp[j] += ev(d.adj_sp[j], env, memo)
        gtr[k] = ev(d.adj_tr, env, memo)
        if k == 0:
            for b in range(m.nu):
                gup[b] = ev(d.adj_up[b], env, memo)
    return gsp, gtr, gup


def expand_patterns(g, y, H, x0, dt, setpoint=(), traj=None, lam=None, lam_d=None, u_prev=None):
    """The same outputs for a pattern model (simd_patterns.generate),
    emulating its kernels: every instance's values go to the per-stage
    scratch at the generated positions, the Jacobian entries to the
    generated slots, and the sums follow the generated lists.  lam: the
    equality rows' multipliers (state and algebraic rows, stage-major),
    lam_d: the inequality rows'.  Also returns the cold-start guess."""
    ders, st = g.pattern_structure
    ns, nx = g.ns, g.nx
    rps, nd = nx + st["n_alg"], st["nd"]
    mc = H * rps
    ncoo = max(st["ncoo"], 1)
    jptr = [0]
    jr, jc = [], []
    for k in range(H):
        for r in range(rps):
            if k > 0:
                for q in range(st["prev_ptr"][r], st["prev_ptr"][r + 1]):
                    jr.append(k * rps + r)
                    jc.append((k - 1) * ns + st["prev_cols"][q])
            for q in range(st["row_ptr"][r], st["row_ptr"][r + 1]):
                jr.append(k * rps + r)
                jc.append(k * ns + st["row_cols"][q])
            jptr.append(len(jr))
    for k in range(H):
        for r in range(nd):
            for q in range(st["ineq_ptr"][r], st["ineq_ptr"][r + 1]):
                jr.append(mc + k * nd + r)
                jc.append(k * ns + st["ineq_cols"][q])
            jptr.append(len(jr))
    jv = np.full(len(jr), np.nan)
    c = np.zeros(H * rps)
    dvals = np.zeros(H * nd)
    grad = np.zeros(H * ns)
    fterm = np.zeros(H * ns)
    nwx = len(st["xlist"])
    Ss = []
    for k in range(H):
        S = np.full(ncoo, np.nan)
        Ss.append(S)
        V = y[k * ns:(k + 1) * ns]
        P = y[(k - 1) * ns:(k - 1) * ns + nx] if k > 0 else x0
        PU = y[(k - 1) * ns + nx:(k - 1) * ns + nx + g.nu] if k > 0 else u_prev
        for pi, dd in enumerate(ders):
            pat = dd.pat
            n = len(pat.instances)
            base = st["coo_base"][pi]
            for i, inst in enumerate(pat.instances):
                env = {("dt", 0): dt, ("tr", 0): 0.0 if traj is None else traj[k]}
                for j, v in enumerate(inst["vars"]):
                    env[("sv", j)] = V[v]
                for j, q in enumerate(inst.get("prevs", [])):
                    env[("sprev", j)] = P[q]
                for j, x in enumerate(inst.get("data", [])):
                    env[("sd", j)] = x
                for j, q in enumerate(inst.get("sps", [])):
                    env[("ssp", j)] = setpoint[q]
                for j, b in enumerate(inst.get("pus", [])):
                    env[("spu", j)] = PU[b]
                memo = {}
                if pat.kind in ("row", "alg", "ineq"):
                    if pat.kind == "ineq":
                        r = k * nd + st["drow"][(pi, i)]
                        dvals[r] = ev(pat.expr, env, memo)
                        row0, off = jptr[mc + r], 0
                        lr = 0.0 if lam_d is None else lam_d[r]
                    else:
                        r = k * rps + (inst["target"] if pat.kind == "row" else st["arow"][(pi, i)])
                        c[r] = ev(pat.expr, env, memo)
                        row0, off = jptr[r], (len(inst.get("prevs", [])) if k > 0 else 0)
                        lr = 0.0 if lam is None else lam[r]
                        if k > 0:
                            for qi, coef in enumerate(dd.pcoef):
                                jv[row0 + st["ppos"][(pi, i)][qi]] = coef
                    for s_, e in enumerate(dd.dv):
                        jv[row0 + off + st["jpos"][(pi, i)][s_]] = ev(e, env, memo)
                    for cc, e in enumerate(dd.d2):
                        S[base + cc * n + i] = lr * ev(e, env, memo)
                else:
                    npair = len(dd.pairs)
                    o_x, o_p, o_g = st["offs"][pi]
                    S[base + (npair + pat.nv) * n + i] = ev(pat.expr, env, memo)
                    for cc, e in enumerate(dd.d2):
                        S[base + cc * n + i] = ev(e, env, memo)
                    for s_, e in enumerate(dd.dv):
                        S[base + (npair + s_) * n + i] = ev(e, env, memo)
                    for cc, e in enumerate(dd.xd2 or []):
                        S[base + (o_x + cc) * n + i] = ev(e, env, memo)
                    for cc, e in enumerate(dd.pd2 or []):
                        S[base + (o_p + cc) * n + i] = ev(e, env, memo)
                    for b, e in enumerate(dd.dpu or []):
                        S[base + (o_g + b) * n + i] = ev(e, env, memo)
    wv, wr, wc = [], [], []
    for k in range(H):
        S = Ss[k]
        Sn = Ss[k + 1] if k + 1 < H else None
        for e, lst in enumerate(st["w_lists"]):
            acc = sum(S[q] for q in lst)
            if Sn is not None:
                acc += sum(Sn[q] for q in st["wn_lists"][e])
            wv.append(acc)
            wr.append(k * ns + g.w_rows[e])
            wc.append(k * ns + g.w_cols[e])
        if k > 0:
            for e, lst in enumerate(st["x_lists"]):
                wv.append(sum(S[q] for q in lst))
                wr.append(k * ns + g.wx_rows[e])
                wc.append((k - 1) * ns + nx + g.wx_cols[e])
        for v in range(ns):
            acc = sum(S[q] for q in st["g_lists"][v])
            if Sn is not None:
                acc += sum(Sn[q] for q in st["gn_lists"][v])
            grad[k * ns + v] = acc
            fterm[k * ns + v] = sum(S[q] for q in st["f_lists"][v])
    wv, wr, wc = np.array(wv), np.array(wr, dtype=int), np.array(wc, dtype=int)
    guess = None
    if u_prev is not None:
        gs = np.zeros(ns)
        gs[:nx] = x0
        gs[nx:nx + g.nu] = u_prev
        m = g.pattern_model
        for gp in m.guesses:
            for inst in gp.instances:
                env = {("dt", 0): dt}
                for j, q in enumerate(inst.get("x0s", [])):
                    env[("sx0", j)] = x0[q]
                for j, q in enumerate(inst.get("ups", [])):
                    env[("sup", j)] = u_prev[q]
                for j, x in enumerate(inst.get("data", [])):
                    env[("sd", j)] = x
                gs[inst["target"]] = ev(gp.expr, env)
        guess = np.tile(gs, H)
    return dict(f=fterm.sum(), grad=grad, c=c, d=dvals, jv=jv, jr=np.array(jr, dtype=int),
                jc=np.array(jc, dtype=int), wv=wv, wr=wr, wc=wc, guess=guess)

