"""Models written with the stage-pattern front end (paper_2606_04725_amd.simd).

Each function returns a StageModel; `simd.compile` turns it into the kernels
the library loads (family NMPC_FAMILY_STAGE_MODEL).

  toy_model        the one-state example of the re-solve listing (Section 3.3):
                   dy/dt = 4 sin(u) - y^3, y >= 0, 1 <= u <= 3, objective
                   dt sum_k (y_k - s_k)^2 with s_k the stage's trajectory value
  lq_model         linear dynamics x_k = A x_{k-1} + B u_k (previous states
                   through a constant matrix), objective
                   sum_k (x_k - xs)^T Q (x_k - xs) + u_k^T R u_k, xs the setpoint
  reflux_model     the distillation case study of Section 4.1 with the
                   algebraic vapour fractions and flows kept as variables
                   (the same problem as the library's REFLUX_COLUMN family)
  distillation_model
                   the workload column (the library's DISTILLATION family):
                   reflux R and boilup V as controls, the equilibrium
                   substituted, feed composition as the stage trajectory,
                   inequality rows for nonnegative distillate and bottoms and
                   a move penalty on the previous stage's controls
  plate_case_model the heated-plate case study of Section 4.2: (n - 2)^2
                   interior temperatures of a grid on [-1, 1]^2 under a
                   5-point Laplacian, heated through the left and bottom edges
                   by the input Q (edge values 4.1 Q^(1/3) and Q^(1/2)),
                   tracking of a region's temperature (trapezoid weights) as
                   the stage trajectory; input in units of q_scale, rows
                   divided by their diagonal coefficient
  plate_pattern_model
                   the workload plate (the library's HEATED_PLATE family)
                   written with index-data patterns: one 5-point stencil
                   row pattern over the G^2 nodes (a neighbour beyond an
                   edge is that edge's heater segment, a control) and one
                   tracking pattern over the nodes with the target field as
                   setpoint
"""
from __future__ import annotations

import numpy as np

from .simd import StageModel, sin
from .simd_patterns import PatternModel


def toy_model() -> StageModel:
    m = StageModel("toy_sin_cube")
    y = m.state("y", lb=0.0)
    u = m.control("u", lb=1.0, ub=3.0)
    m.dynamics(y, 4.0 * sin(u) - y ** 3)
    m.minimize(m.dt * (y - m.traj()) ** 2)
    m.guess(u, 2.0)
    return m


def lq_model(A, B, Q, R, name="lq", x_bounds=None, u_bounds=None) -> StageModel:
    A, B, Q, R = (np.asarray(v, dtype=np.float64) for v in (A, B, Q, R))
    nx, nu = B.shape
    m = StageModel(name, n_setpoint=nx)
    xl, xh = x_bounds if x_bounds is not None else (-np.inf, np.inf)
    ul, uh = u_bounds if u_bounds is not None else (-np.inf, np.inf)
    X = [m.state(f"x{i}", xl, xh) for i in range(nx)]
    U = [m.control(f"u{j}", ul, uh) for j in range(nu)]
    for i in range(nx):
        r = X[i]
        for j in range(nx):
            if A[i, j] != 0.0:
                r = r - float(A[i, j]) * m.prev(X[j])
        for j in range(nu):
            if B[i, j] != 0.0:
                r = r - float(B[i, j]) * U[j]
        m.state_equation(X[i], r)
    E = [X[i] - m.setpoint(i) for i in range(nx)]
    f = 0.0
    for i in range(nx):
        for j in range(nx):
            if Q[i, j] != 0.0:
                f = f + float(Q[i, j]) * E[i] * E[j]
    for i in range(nu):
        for j in range(nu):
            if R[i, j] != 0.0:
                f = f + float(R[i, j]) * U[i] * U[j]
    m.minimize(f)
    for j in range(nu):
        m.guess(U[j], 0.0)
    return m


def reflux_model(N=32, Nf=17, D=0.2, F=0.4, alpha=1.6, xf=0.5, Ac=0.5, At=0.25, Ar=1.0, w_u=0.1,
                 x_lo=0.0, x_hi=1.0, u_lo=1.0, u_hi=5.0, flow_hi=10.0) -> StageModel:
    """Setpoint (xbar, ubar): tracking of the condenser composition and the
    reflux ratio; stage layout [x_1..x_N, u, y_1..y_N, L, V, S]."""
    m = StageModel(f"reflux_N{N}_Nf{Nf}", n_setpoint=2)
    x = [None] + [m.state(f"x{i}", x_lo, x_hi) for i in range(1, N + 1)]
    u = m.control("u", u_lo, u_hi)
    y = [None] + [m.algebraic_var(f"y{i}", x_lo, x_hi) for i in range(1, N + 1)]
    L = m.algebraic_var("L", 0.0, flow_hi)
    V = m.algebraic_var("V", 0.0, flow_hi)
    S = m.algebraic_var("S", 0.0, flow_hi)
    m.dynamics(x[1], V * (y[2] - x[1]) / Ac)
    for i in range(2, N):
        lin = L if i <= Nf else S
        lout = L if i < Nf else S
        f = lin * x[i - 1] - lout * x[i] - V * (y[i] - y[i + 1])
        if i == Nf:
            f = f + F * xf
        m.dynamics(x[i], f / At)
    m.dynamics(x[N], (S * x[N - 1] - (F - D) * x[N] - V * y[N]) / Ar)
    for i in range(1, N + 1):
        m.equality(y[i] - alpha * x[i] / (1.0 + (alpha - 1.0) * x[i]))
    m.equality(L - u * D)
    m.equality(V - L - D)
    m.equality(S - L - F)
    m.minimize(m.dt * ((x[1] - m.setpoint(0)) ** 2 + w_u * (u - m.setpoint(1)) ** 2))
    # cold start: measured trays, last reflux ratio, its equilibrium vapour and flows
    up = m.u_prev(0)
    for i in range(1, N + 1):
        xi = m.x0(i - 1)
        m.guess(y[i], alpha * xi / (1.0 + (alpha - 1.0) * xi))
    m.guess(L, up * D)
    m.guess(V, up * D + D)
    m.guess(S, up * D + F)
    return m


def distillation_model(N, alpha, F=1.0, rho=1e-2, x_lo=0.0, x_hi=1.0, u_lo=0.5, u_hi=5.0) -> StageModel:
    """States x_0 (condenser) .. x_{N+1} (reboiler), controls (R, V), feed on
    tray N // 2 with composition the stage's trajectory value; objective
    (x_0 - xD*)^2 + (x_{N+1} - xB*)^2 + rho |u - u_prev|^2 per stage with
    (xD*, xB*) the setpoint; R - V <= 0 and V - R - F <= 0."""
    m = StageModel(f"distillation_N{N}", n_setpoint=2)
    x = [m.state(f"x{i}", x_lo, x_hi) for i in range(N + 2)]
    R = m.control("R", u_lo, u_hi)
    V = m.control("V", u_lo, u_hi)
    fd = N // 2
    zF = m.traj()

    def vle(xi):
        return alpha * xi / (1.0 + (alpha - 1.0) * xi)

    m.dynamics(x[0], V * (vle(x[1]) - x[0]))
    for i in range(1, N + 1):
        lin = R if i <= fd else R + F
        lout = R if i < fd else R + F
        f = lin * x[i - 1] - lout * x[i] + V * (vle(x[i + 1]) - vle(x[i]))
        if i == fd:
            f = f + F * zF
        m.dynamics(x[i], f)
    m.dynamics(x[N + 1], (R + F) * x[N] - V * vle(x[N + 1]) - (R + F - V) * x[N + 1])
    m.inequality(R - V)
    m.inequality(V - R - F)
    m.minimize((x[0] - m.setpoint(0)) ** 2 + (x[N + 1] - m.setpoint(1)) ** 2
               + rho * ((R - m.prev_control(R)) ** 2 + (V - m.prev_control(V)) ** 2))
    return m


def plate_case_model(n=21, alpha=230.0, Tb=50.0, loss=50.0, rho=1e-8, Q_lo=50.0, q_scale=1e4,
                     dt=0.08) -> StageModel:
    """Stage layout [T at the interior points (x1 fastest), q = Q / q_scale];
    rows rs (T - T_prev - dt alpha (lap_h T - loss)) with rs = 1 / (1 + 4 dt
    alpha / h^2); objective dt (sum_p w_p (T_p - T_sp)^2 + rho Q^2) with the
    tracked temperature T_sp the stage's trajectory value and w_p the
    trapezoid weights of [-0.5, 0.5]^2.  The stage length is a number of the
    model here (the row scale depends on it): create the structure with the
    same dt."""
    g = n - 2
    h = 2.0 / (n - 1)
    rs = 1.0 / (1.0 + 4.0 * dt * alpha / (h * h))
    m = StageModel(f"plate_case_n{n}")
    T = [m.state(f"T{p}") for p in range(g * g)]
    q = m.control("q", lb=Q_lo / q_scale)
    Q = q_scale * q
    left, bottom = 4.1 * Q ** (1.0 / 3.0), Q ** 0.5
    for j in range(g):
        for i in range(g):
            p = j * g + i
            west = T[p - 1] if i > 0 else left
            east = T[p + 1] if i < g - 1 else Tb
            south = T[p - g] if j > 0 else bottom
            north = T[p + g] if j < g - 1 else Tb
            lap = (west + east + south + north - 4.0 * T[p]) * (1.0 / (h * h))
            m.state_equation(T[p], rs * (T[p] - m.prev(T[p])) - (rs * dt * alpha) * (lap - loss))
    coord = [-1.0 + h * (i + 1) for i in range(g)]

    def weight(x):
        if abs(x) > 0.5 + 1e-12:
            return 0.0
        return 0.5 if abs(abs(x) - 0.5) < 1e-12 else 1.0

    track = 0.0
    for j in range(g):
        for i in range(g):
            wgt = weight(coord[i]) * weight(coord[j])
            if wgt:
                track = track + (h * h * wgt) * (T[j * g + i] - m.traj()) ** 2
    m.minimize(dt * (track + rho * Q * Q))
    return m


def plate_pattern_model(G, sigma=0.1, t_hi=1.5, c_lo=0.0, c_hi=1.0) -> PatternModel:
    """The plate of eq. (3)'s repeated pattern: G x G interior nodes at
    spacing h = 1 / (G + 1), node p = b G + a; conductivity 1 + sigma T with
    the face average, so the flux from a neighbour v into T is
    [(v - T) + (sigma / 2)(v^2 - T^2)] / h^2; backward Euler in time.  The
    four neighbours in the order below, left, right, above; one beyond an
    edge is the heater segment of that edge covering the node (edges bottom,
    right, top, left, 4 segments of G / 4 nodes each, segment 4 edge +
    coordinate // (G / 4)).  Objective: sum over nodes of (T_p - T*_p)^2, T*
    the setpoint field.  Bounds T <= t_hi, c_lo <= u <= c_hi."""
    if G % 4 or G < 4:
        raise ValueError("the grid size must be a positive multiple of 4")
    m = PatternModel(f"plate_pattern_G{G}", n_setpoint=G * G)
    T = m.states(G * G, ub=t_hi)
    U = m.controls(16, lb=c_lo, ub=c_hi)
    q = G // 4
    kap, inv_h2 = 0.5 * sigma, float((G + 1) * (G + 1))

    def neighbours(a, b):
        return [T[(b - 1) * G + a] if b > 0 else U[0 * 4 + a // q],
                T[b * G + a - 1] if a > 0 else U[3 * 4 + b // q],
                T[b * G + a + 1] if a < G - 1 else U[1 * 4 + b // q],
                T[(b + 1) * G + a] if b < G - 1 else U[2 * 4 + a // q]]

    def stencil(v, p, d):
        t = v[0]
        flux = sum(((n - t) + kap * (n * n - t * t) for n in v[1:]), 0.0)
        return t - p[0] - m.dt * inv_h2 * flux

    rows = [dict(target=T[b * G + a], vars=[T[b * G + a]] + neighbours(a, b), prevs=[T[b * G + a]])
            for b in range(G) for a in range(G)]
    m.row_pattern(stencil, rows, nv=5, nprev=1)
    m.objective_pattern(lambda v, d, s: (v[0] - s[0]) ** 2,
                        [dict(vars=[T[p]], sps=[p]) for p in range(G * G)], nv=1, nsp=1)
    return m


def plate_case_pattern_model(n=21, alpha=230.0, Tb=50.0, loss=50.0, rho=1e-8, Q_lo=50.0, q_scale=1e4,
                             dt=0.08) -> PatternModel:
    """The heated-plate case study (the same problem as plate_case_model)
    written with index-data patterns: one row pattern per kind of grid point
    (interior; an edge point next to a heated edge, the heater's edge function
    chosen by instance data; next to an unheated edge; the four corner kinds)
    and two objective patterns (the tracking term of a weighted point, the
    input cost).  Stage layout [T at the interior points (x1 fastest), q]."""
    g = n - 2
    h = 2.0 / (n - 1)
    inv_h2 = 1.0 / (h * h)
    rs = 1.0 / (1.0 + 4.0 * dt * alpha * inv_h2)
    m = PatternModel(f"plate_case_pattern_n{n}")
    T = m.states(g * g)
    (q,) = m.controls(1, lb=Q_lo / q_scale)

    def left(v):
        return 4.1 * (q_scale * v) ** (1.0 / 3.0)

    def bottom(v):
        return (q_scale * v) ** 0.5

    def row(t, prev, nbr_sum):
        lap = (nbr_sum - 4.0 * t) * inv_h2
        return rs * (t - prev) - (rs * dt * alpha) * (lap - loss)

    kinds = {}   # kind -> list of instances
    for j in range(g):
        for i in range(g):
            p = j * g + i
            nb, heat, cold = [], [], 0
            if i > 0:
                nb.append(T[p - 1])
            else:
                heat.append(0)            # west: the left heater
            if i < g - 1:
                nb.append(T[p + 1])
            else:
                cold += 1                 # east: Tb
            if j > 0:
                nb.append(T[p - g])
            else:
                heat.append(1)            # south: the bottom heater
            if j < g - 1:
                nb.append(T[p + g])
            else:
                cold += 1                 # north: Tb
            inst = dict(target=T[p], vars=[T[p]] + nb + ([q] if heat else []), prevs=[T[p]],
                        data=[1.0 if 0 in heat else 0.0, 1.0 if 1 in heat else 0.0])
            kinds.setdefault((len(nb), len(heat), cold), []).append(inst)
    for (nn, nh, nc), insts in sorted(kinds.items()):
        def tmpl(v, p, d, nn=nn, nh=nh, nc=nc):
            s = sum(v[1:1 + nn], 0.0) + nc * Tb
            if nh:
                s = s + d[0] * left(v[1 + nn]) + d[1] * bottom(v[1 + nn])
            return row(v[0], p[0], s)
        m.row_pattern(tmpl, insts, nv=1 + nn + (1 if nh else 0), nprev=1, ndata=2)
    coord = [-1.0 + h * (i + 1) for i in range(g)]

    def weight(x):
        if abs(x) > 0.5 + 1e-12:
            return 0.0
        return 0.5 if abs(abs(x) - 0.5) < 1e-12 else 1.0

    track = [dict(vars=[T[j * g + i]], data=[h * h * weight(coord[i]) * weight(coord[j])])
             for j in range(g) for i in range(g) if weight(coord[i]) * weight(coord[j])]
    tr = m.traj()
    m.objective_pattern(lambda v, d, s: dt * d[0] * (v[0] - tr) ** 2, track, nv=1, ndata=1)
    m.objective_pattern(lambda v, d, s: (dt * rho * q_scale * q_scale) * v[0] * v[0], [dict(vars=[q])], nv=1)
    return m


def reflux_pattern_model(N=32, Nf=17, D=0.2, F=0.4, alpha=1.6, xf=0.5, Ac=0.5, At=0.25, Ar=1.0, w_u=0.1,
                         x_lo=0.0, x_hi=1.0, u_lo=1.0, u_hi=5.0, flow_hi=10.0) -> PatternModel:
    """The distillation case study (the same problem as reflux_model) written
    with index-data patterns: a tray pattern (the liquid flow slot bound to L
    above the feed and S below it), the feed tray, condenser and reboiler;
    the equilibrium as one algebraic pattern over the trays and the three
    flow balances; tracking of the condenser and the reflux ratio; guesses of
    the vapour fractions and flows from the measured trays and the last
    reflux ratio.  Stage layout [x_1..x_N, u, y_1..y_N, L, V, S]."""
    m = PatternModel(f"reflux_pattern_N{N}_Nf{Nf}", n_setpoint=2)
    x = [None] + m.states(N, x_lo, x_hi)
    (u,) = m.controls(1, u_lo, u_hi)
    y = [None] + m.algebraic(N, x_lo, x_hi)
    L, V, S = m.algebraic(3, 0.0, flow_hi)
    dt = m.dt

    def euler(v, p, f):
        return v[0] - p[0] - dt * f

    # condenser: V (y_2 - x_1) / Ac
    m.row_pattern(lambda v, p, d: euler(v, p, v[1] * (v[2] - v[0]) / Ac),
                  [dict(target=x[1], vars=[x[1], V, y[2]], prevs=[x[1]])], nv=3, nprev=1)
    # trays other than the feed: Fl (x_{i-1} - x_i) - V (y_i - y_{i+1}), Fl = L above the feed, S below
    trays = [dict(target=x[i], vars=[x[i], L if i < Nf else S, x[i - 1], V, y[i], y[i + 1]], prevs=[x[i]])
             for i in range(2, N) if i != Nf]
    m.row_pattern(lambda v, p, d: euler(v, p, (v[1] * (v[2] - v[0]) - v[3] * (v[4] - v[5])) / At),
                  trays, nv=6, nprev=1)
    # feed tray: L x_{i-1} - S x_i - V (y_i - y_{i+1}) + F xf
    m.row_pattern(lambda v, p, d: euler(v, p, (v[1] * v[3] - v[2] * v[0] - v[4] * (v[5] - v[6]) + F * xf) / At),
                  [dict(target=x[Nf], vars=[x[Nf], L, S, x[Nf - 1], V, y[Nf], y[Nf + 1]], prevs=[x[Nf]])],
                  nv=7, nprev=1)
    # reboiler: S x_{N-1} - (F - D) x_N - V y_N
    m.row_pattern(lambda v, p, d: euler(v, p, (v[1] * v[2] - (F - D) * v[0] - v[3] * v[4]) / Ar),
                  [dict(target=x[N], vars=[x[N], S, x[N - 1], V, y[N]], prevs=[x[N]])], nv=5, nprev=1)
    m.algebraic_row_pattern(lambda v, d: v[0] - alpha * v[1] / (1.0 + (alpha - 1.0) * v[1]),
                            [dict(vars=[y[i], x[i]]) for i in range(1, N + 1)], nv=2)
    m.algebraic_row_pattern(lambda v, d: v[0] - v[1] * D, [dict(vars=[L, u])], nv=2)
    m.algebraic_row_pattern(lambda v, d: v[0] - v[1] - D, [dict(vars=[V, L])], nv=2)
    m.algebraic_row_pattern(lambda v, d: v[0] - v[1] - F, [dict(vars=[S, L])], nv=2)
    m.objective_pattern(lambda v, d, s: dt * ((v[0] - s[0]) ** 2 + w_u * (v[1] - s[1]) ** 2),
                        [dict(vars=[x[1], u], sps=[0, 1])], nv=2, nsp=2)
    m.guess_pattern(lambda xs, us, d: alpha * xs[0] / (1.0 + (alpha - 1.0) * xs[0]),
                    [dict(target=y[i], x0s=[x[i]]) for i in range(1, N + 1)], nx0=1)
    m.guess_pattern(lambda xs, us, d: us[0] * D + d[0],
                    [dict(target=L, ups=[0], data=[0.0]), dict(target=V, ups=[0], data=[D]),
                     dict(target=S, ups=[0], data=[F])], nup=1, ndata=1)
    return m


def row_kinds_model() -> PatternModel:
    """A small pattern model with every row kind: two state rows, an
    algebraic row, two inequality rows, an objective and a guess pattern
    (stage layout [x0, x1, u0, u1, a]); the tests compare its generated kernels
    with the host evaluation of the same expressions."""
    m = PatternModel("row_kinds")
    X = m.states(2)
    U = m.controls(2, lb=-1.0, ub=1.0)
    (A,) = m.algebraic(1)
    m.row_pattern(lambda v, p, d: v[0] - p[0] - m.dt * v[1] * v[1],
                  [dict(target=X[j], vars=[X[j], U[j]], prevs=[X[j]]) for j in range(2)], nv=2, nprev=1)
    m.algebraic_row_pattern(lambda v, d: v[0] - v[1] * v[2], [dict(vars=[A, X[0], X[1]])], nv=3)
    m.inequality_pattern(lambda v, d: d[0] * v[0] * v[0] + v[1] - d[1],
                         [dict(vars=[U[0], X[1]], data=[2.0, 1.0]), dict(vars=[U[1], A], data=[0.5, 3.0])],
                         nv=2, ndata=2)
    m.objective_pattern(lambda v, d, s: (v[0] - 1.0) ** 2 + v[1] ** 2, [dict(vars=[X[0], A])], nv=2)
    m.guess_pattern(lambda x, u, d: x[0] * x[1] + d[0], [dict(target=A, x0s=[0, 1], data=[0.25])], nx0=2,
                    ndata=1)
    return m


def distillation_pattern_model(N, alpha, F=1.0, rho=1e-2, x_lo=0.0, x_hi=1.0, u_lo=0.5, u_hi=5.0) -> PatternModel:
    """The workload column (the same problem as distillation_model and the
    library's DISTILLATION family) written with index-data patterns: one tray
    pattern over the trays other than the feed tray (liquid flow R above the
    feed, R + F below it, chosen by instance data), the feed tray (which reads
    the stage's feed composition), condenser and reboiler; both flow
    inequalities as one pattern; the objective with the move penalty in the
    previous stage's controls.  Stage layout [x_0 .. x_{N+1}, R, V]."""
    m = PatternModel(f"distillation_pattern_N{N}", n_setpoint=2)
    x = m.states(N + 2, x_lo, x_hi)
    R, V = m.controls(2, u_lo, u_hi)
    fd = N // 2
    dt, zF = m.dt, m.traj()

    def vle(xi):
        return alpha * xi / (1.0 + (alpha - 1.0) * xi)

    def euler(v, p, f):
        return v[0] - p[0] - dt * f

    m.row_pattern(lambda v, p, d: euler(v, p, v[1] * (vle(v[2]) - v[0])),
                  [dict(target=x[0], vars=[x[0], V, x[1]], prevs=[x[0]])], nv=3, nprev=1)
    # trays i != fd: (R + d0) (x_{i-1} - x_i) + V (vle(x_{i+1}) - vle(x_i)), d0 = 0 above the feed, F below
    trays = [dict(target=x[i], vars=[x[i], R, V, x[i - 1], x[i + 1]], prevs=[x[i]], data=[0.0 if i < fd else F])
             for i in range(1, N + 1) if i != fd]
    m.row_pattern(lambda v, p, d: euler(v, p, (v[1] + d[0]) * (v[3] - v[0]) + v[2] * (vle(v[4]) - vle(v[0]))),
                  trays, nv=5, nprev=1, ndata=1)
    m.row_pattern(lambda v, p, d: euler(v, p, v[1] * v[3] - (v[1] + F) * v[0] + v[2] * (vle(v[4]) - vle(v[0]))
                                        + F * zF),
                  [dict(target=x[fd], vars=[x[fd], R, V, x[fd - 1], x[fd + 1]], prevs=[x[fd]])], nv=5, nprev=1)
    m.row_pattern(lambda v, p, d: euler(v, p, (v[1] + F) * v[3] - v[2] * vle(v[0]) - (v[1] + F - v[2]) * v[0]),
                  [dict(target=x[N + 1], vars=[x[N + 1], R, V, x[N]], prevs=[x[N + 1]])], nv=4, nprev=1)
    m.inequality_pattern(lambda v, d: v[0] - v[1] - d[0], [dict(vars=[R, V], data=[0.0]),
                                                           dict(vars=[V, R], data=[F])], nv=2, ndata=1)
    m.objective_pattern(lambda v, d, s, pu: (v[0] - s[0]) ** 2 + (v[1] - s[1]) ** 2
                        + rho * ((v[2] - pu[0]) ** 2 + (v[3] - pu[1]) ** 2),
                        [dict(vars=[x[0], x[N + 1], R, V], sps=[0, 1], pus=[0, 1])], nv=4, nsp=2, npu=2)
    return m
