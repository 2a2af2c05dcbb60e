"""Pins for the oracle's Lifted-KKT interior-point method (Section 3.2)."""
import numpy as np
import pytest
import scipy.optimize as so

from oracle.distillation import DistillationOCP
from oracle.ipm import LiftedIPM, IPMOptions, CholeskySolver
from oracle.kkt import kkt_error
from oracle.lq import LQOCP, random_lq
from oracle.riccati import riccati_solution, riccati_gains
from oracle.toy import ToyOCP
from oracle.nmpc import distillation_episode
from workloads import distillation_workload


def _cold(ipm, m):
    st = ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold)
    return ipm.solve(st, ipm.o.mu0_cold)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lq_matches_riccati(seed):
    A, B, Q, R, x0, xs = random_lq(4, 2, 12, seed=seed)
    m = LQOCP(A, B, Q, R, 12, xs=xs)
    m.set_parameters(x0=x0)
    ipm = LiftedIPM(m)
    res = _cold(ipm, m)
    assert res.status == 0
    X, U = riccati_solution(A, B, Q, R, 12, x0, xs)
    Y = res.state.y.reshape(12, 6)
    scale = max(1.0, np.max(np.abs(U)))
    assert np.max(np.abs(Y[:, 4:] - U)) <= 1e-6 * scale
    assert np.max(np.abs(Y[:, :4] - X)) <= 1e-6 * max(1.0, np.max(np.abs(X)))
    # first-stage gain: u_1* is affine in x0 with slope -K_1
    K, _ = riccati_gains(A, B, Q, R, 12, xs)
    dx = np.zeros(4)
    dx[0] = 1e-3
    m.set_parameters(x0=x0 + dx)
    res2 = _cold(LiftedIPM(m), m)
    du = (res2.state.y[4:6] - res.state.y[4:6]) / 1e-3
    assert np.allclose(du, -K[1][:, 0], rtol=1e-4, atol=1e-5)


def test_toy_matches_scipy():
    m = ToyOCP()
    m.set_parameters(y0=1.0, tk=0.0)
    ipm = LiftedIPM(m)
    res = _cold(ipm, m)
    assert res.status == 0
    bounds = list(zip(m.lb, [u if np.isfinite(u) else None for u in m.ub]))
    sol = so.minimize(m.f, m.initial_guess(), jac=m.grad, method="SLSQP",
                      constraints=[{"type": "eq", "fun": m.cons_c, "jac": lambda y: m.jac_c(y).toarray()}],
                      bounds=bounds, options={"ftol": 1e-12, "maxiter": 1000})
    assert sol.success
    # several controls sit on their upper bound 3; the barrier keeps them mu/z away
    assert np.max(np.abs(sol.x - res.state.y)) < 1e-6
    assert abs(sol.fun - m.f(res.state.y)) < 1e-7


def test_distillation_episode_kkt():
    w = distillation_workload("small", 4)
    m, out = distillation_episode(w)
    for o in out:
        assert o["status"] == 0
        m.set_parameters(x0=o["x0"], zF=o["zF"], u_prev=o["u_prev"])
        e = kkt_error(m, o["y"], o["lam"], o["omega_d"], o["zL"], o["zU"])
        assert e["max"] <= 1e-8, e
    # warm re-solves need far fewer iterations than the cold first solve
    assert max(o["iters"] for o in out[1:]) < out[0]["iters"]


def _full_newton(ipm, st, mu, gf, c, d, Jc, Jd, W):
    """Unreduced primal-dual Newton system of the lifted barrier problem, solved
    densely: unknowns (dy, ds, domega, dbeta, dzL, dzU)."""
    n, ml = ipm.n, ipm.ml
    G = np.vstack([Jc.toarray(), -Jc.toarray()] + ([Jd.toarray()] if ipm.md else []))
    gL, gU = ipm.gaps(st.y)
    hL, hU = ipm.hasL.astype(float), ipm.hasU.astype(float)
    N = 2 * n + 3 * ml + n
    iy, is_, iw, ib, iL, iU = 0, n, n + ml, n + 2 * ml, n + 3 * ml, 2 * n + 3 * ml
    M = np.zeros((N, N))
    r = np.zeros(N)
    M[iy:iy + n, iy:iy + n] = W.toarray()
    M[iy:iy + n, iw:iw + ml] = G.T
    M[iy:iy + n, iL:iL + n] = -np.eye(n)
    M[iy:iy + n, iU:iU + n] = np.eye(n)
    r[iy:iy + n] = -(gf + G.T @ st.omega - st.zL + st.zU)
    M[is_:is_ + ml, iw:iw + ml] = np.eye(ml)
    M[is_:is_ + ml, ib:ib + ml] = -np.eye(ml)
    r[is_:is_ + ml] = -(st.omega - st.beta)
    M[iw:iw + ml, iy:iy + n] = G
    M[iw:iw + ml, is_:is_ + ml] = np.eye(ml)
    r[iw:iw + ml] = -(ipm.g_lifted(c, d) + st.s)
    M[ib:ib + ml, is_:is_ + ml] = np.diag(st.beta)
    M[ib:ib + ml, ib:ib + ml] = np.diag(st.s)
    r[ib:ib + ml] = mu - st.s * st.beta
    M[iL:iL + n, iy:iy + n] = np.diag(st.zL * hL)
    M[iL:iL + n, iL:iL + n] = np.diag(np.where(ipm.hasL, gL, 1.0))
    r[iL:iL + n] = hL * (mu - gL * st.zL)
    M[iU:iU + n, iy:iy + n] = -np.diag(st.zU * hU)
    M[iU:iU + n, iU:iU + n] = np.diag(np.where(ipm.hasU, gU, 1.0))
    r[iU:iU + n] = hU * (mu - gU * st.zU)
    x = np.linalg.solve(M, r)
    return dict(dy=x[iy:iy + n], ds=x[is_:is_ + ml], domega=x[iw:iw + ml], dbeta=x[ib:ib + ml],
                dzL=x[iL:iL + n], dzU=x[iU:iU + n])


@pytest.mark.parametrize("mu", [1e-1, 1e-3])
def test_condensation_matches_full_newton(mu):
    """eq. (14)/(17): the condensed solve gives the same direction as the full
    augmented Newton system (eq. 10 with bounds), at an interior point."""
    m = DistillationOCP(3, 3, 0.1, 2.5)
    w = distillation_workload("small", 0, N=3, H=3)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), 0.1)
    rng = np.random.default_rng(0)
    st.omega = rng.normal(size=ipm.ml)
    f, gf = m.f(st.y), m.grad(st.y)
    c, d = m.cons_c(st.y), m.cons_d(st.y)
    Jc, Jd = m.jac_c(st.y), m.jac_d(st.y)
    step = ipm.newton_step(st, mu, f, gf, c, d, Jc, Jd)
    if step["eta"] != 0.0:
        pytest.skip("regularized step; identity holds only for eta = 0")
    full = _full_newton(ipm, st, mu, gf, c, d, Jc, Jd, step["W"])
    for k in ("dy", "ds", "domega", "dbeta", "dzL", "dzU"):
        ref = full[k]
        assert np.max(np.abs(step[k] - ref)) <= 1e-9 * max(1.0, np.max(np.abs(ref))), k


@pytest.mark.parametrize("seed", range(6))
def test_inertia_relation(seed):
    """eq. (15) for the lifted system: K_c = W + Sigma + G^T Q G is positive
    definite iff the lifted augmented matrix [[W+Sigma, 0, G^T], [0, Q, I],
    [G, I, 0]] has inertia (n + m^l, 0, m^l)."""
    rng = np.random.default_rng(seed)
    n, ml = 6, 5
    M = rng.normal(size=(n, n))
    W = (M + M.T) / 2 - rng.uniform(0, 3) * np.eye(n)
    G = rng.normal(size=(ml, n))
    Q = np.diag(rng.uniform(0.01, 2.0, ml))
    Kc = W + G.T @ Q @ G
    Kaug = np.block([[W, np.zeros((n, ml)), G.T],
                     [np.zeros((ml, n)), Q, np.eye(ml)],
                     [G, np.eye(ml), np.zeros((ml, ml))]])
    ev = np.linalg.eigvalsh(Kaug)
    good = (np.sum(ev > 1e-10) == n + ml) and (np.sum(ev < -1e-10) == ml)
    chol = CholeskySolver(n, [0], [0])
    chol.banded = False
    assert chol.factor(__import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix(Kc)) == good


def test_cholesky_solver_banded_vs_dense():
    import scipy.sparse as sp
    rng = np.random.default_rng(1)
    n, bw = 60, 4
    A = np.zeros((n, n))
    for k in range(bw + 1):
        v = rng.normal(size=n - k)
        A += np.diag(v, -k)
    K = A @ A.T + 0.1 * np.eye(n)
    rows, cols = np.nonzero(np.tril(K))
    cs = CholeskySolver(n, rows, cols)
    assert cs.banded
    b = rng.normal(size=n)
    assert cs.factor(sp.csr_matrix(K))
    x = cs.solve(b)
    assert np.allclose(K @ x, b, atol=1e-10)
    Kbad = K.copy()
    Kbad[5, 5] = -1.0
    assert not cs.factor(sp.csr_matrix(Kbad))


def test_inertia_correction_path():
    """Indefinite stage cost: the first factorizations fail, eta > 0 is used and
    the method still converges to the KKT point of the (nonconvex) problem."""
    A, B, Q, R, x0, xs = random_lq(3, 2, 6, seed=5, indefinite=True)
    m = LQOCP(A, B, Q, R, 6, xs=xs, x_bounds=(-3.0, 3.0), u_bounds=(-2.0, 2.0))
    m.set_parameters(x0=x0)
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold)
    res = ipm.solve(st, ipm.o.mu0_cold, record=True)
    assert res.status == 0
    assert any(t["eta"] > 0 for t in res.trace)
    lam, om = ipm.multipliers(res.state)
    e = kkt_error(m, res.state.y, lam, om, res.state.zL, res.state.zU)
    assert e["max"] <= 1e-8


@pytest.mark.parametrize("seed", [0, 2])
def test_medium_cold_solve_converges(seed):
    """The benchmark's 40-tray, 100-stage column: the filter line search with
    second-order corrections converges from the cold start to the tolerance."""
    from oracle.distillation import DistillationOCP
    w = distillation_workload("medium", seed)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0 and res.iters <= 60
    st = res.state
    lam = st.omega[:m.m_c] - st.omega[m.m_c:2 * m.m_c]
    assert kkt_error(m, st.y, lam, st.omega[2 * m.m_c:], st.zL, st.zU)["max"] <= 1e-8


def test_merit_fallback_rescues_filter_stall():
    """A ragged-batch column (22 trays, 45 stages) on which the filter search
    stalls: the Newton direction ascends phi while theta barely moves, so every
    trial down to the minimal step is rejected.  Without the fallback the solve
    ends in a line-search failure; with it one l1-merit step gets through, the
    filter restarts empty and the solve reaches a KKT point of the original
    problem."""
    from workloads import batch_distillation_workloads
    w = batch_distillation_workloads(64, 1000)[7]
    assert (w.N, w.H) == (22, 45)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    off = LiftedIPM(m, IPMOptions(merit_fallback=0))
    r0 = off.solve(off.cold_start(m.initial_guess(), off.o.mu0_cold), off.o.mu0_cold)
    assert r0.status == 2
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold, record=True)
    assert res.status == 0
    used = [t["it"] for t in res.trace if t["merit"]]
    assert len(used) >= 1 and used[0] == r0.iters
    st = res.state
    lam = st.omega[:m.m_c] - st.omega[m.m_c:2 * m.m_c]
    assert kkt_error(m, st.y, lam, st.omega[2 * m.m_c:], st.zL, st.zU)["max"] <= 1e-8
