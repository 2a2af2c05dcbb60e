"""GPU parity of the heated-plate family (the second NMPC family) against the
CPU oracle, through the C ABI: model evaluation, the supernodal factorization
and solves on every supernode class the plate's fronts fall into (shared
memory, one workgroup with a global front, and the multi-workgroup path for
large fronts), whole interior-point solves, the sensitivities, and the
32 x 32 x 50 workload at full size (condensed matrix and optimality error
recomputed by the oracle)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import symbolic as S
from oracle.adjoint import sensitivities
from oracle.ipm import LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate import PlateOCP
from paper_2606_04725_amd import nmpc as N
from workloads import plate_workload
from plate_parity import PARITY_TOL, close, note, solve_pair, tighten_gpu, tighten_ref

pytestmark = pytest.mark.gpu


_note = note
_close = close


def _opts(**kw):
    from oracle.ipm import IPMOptions
    return IPMOptions(tol=PARITY_TOL, **kw)


def _pair(G, H, seed=0, ordering=N.capi.NMPC_ORDER_NESTED_DISSECTION):
    w = plate_workload("large", seed, G=G, H=H)
    m = PlateOCP.from_workload(w)
    p = N.Problem(N.plate_structure(G, H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi, ordering=ordering))
    p.analyze()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    return w, m, p


def test_plate_eval_matches_oracle():
    _note("plate eval G=8 H=3")
    w, m, p = _pair(8, 3)
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 1.0, m.n)
    lam = rng.normal(size=m.m_c)
    out = p.eval(y, lam, np.zeros(0))
    pat = p.patterns()
    assert abs(out["f"] - m.f(y)) <= 1e-13 * max(1.0, abs(m.f(y)))
    assert _close(out["grad"], m.grad(y), 1e-13)
    assert _close(out["c"], m.cons_c(y), 1e-13)
    J = m.jac_c(y).tocsr()
    assert _close(out["j_vals"], np.asarray(J[pat["j_rows"], pat["j_cols"]]).ravel(), 1e-13)
    W = m.hess(y, lam, np.zeros(0)).tocsr()
    assert _close(out["w_vals"], np.asarray(W[pat["w_rows"], pat["w_cols"]]).ravel(), 1e-13)


def _kkt_at_cold_start(m, mu=0.1, seed=0):
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), mu)
    st.omega = np.random.default_rng(seed).normal(scale=0.5, size=ipm.ml)
    step = ipm.newton_step(st, mu, m.f(st.y), m.grad(st.y), m.cons_c(st.y), m.cons_d(st.y), m.jac_c(st.y),
                           m.jac_d(st.y))
    return ipm, st, step


@pytest.mark.parametrize("ordering", [N.capi.NMPC_ORDER_NESTED_DISSECTION, N.capi.NMPC_ORDER_FAMILY_DISSECTION])
@pytest.mark.parametrize("G,H", [(8, 4), (16, 10)])
def test_plate_factor_and_solve_match_dense_cholesky(G, H, ordering):
    """16 x 16 x 10 has fronts of every class (up to 416 rows and 256
    columns under the family dissection, 410 rows and 250 columns under the
    default)."""
    _note(f"plate factor G={G} H={H} ordering={ordering}")
    w, m, p = _pair(G, H, ordering=ordering)
    ipm, st, step = _kkt_at_cold_start(m)
    K = (step["K"] + step["eta"] * sp.identity(m.n)).tocsr()
    pat = p.patterns()
    kv = np.asarray(step["K"].tocsr()[pat["k_rows"], pat["k_cols"]]).ravel()
    ok, lv = p.factor(kv, step["eta"])
    assert ok
    sym = p.export_symbolic()
    n = p.n
    Ld = np.zeros((n, n))
    off = 0
    sp_, rp, rows = sym["snode_ptr"], sym["snode_rows_ptr"], sym["snode_rows"]
    for s in range(sym["n_supernodes"]):
        f, l = sp_[s], sp_[s + 1]
        R = rows[rp[s]:rp[s + 1]]
        mr, wd = len(R), l - f
        panel = lv[off:off + mr * wd].reshape(wd, mr).T
        off += mr * wd
        for j in range(wd):
            Ld[R[j:], f + j] = panel[j:, j]
    perm = sym["perm"]
    Lref = np.linalg.cholesky(K.toarray()[np.ix_(perm, perm)])
    assert np.linalg.norm(Ld - Lref) / np.linalg.norm(Lref) <= 1e-12
    rng = np.random.default_rng(2)
    b = rng.normal(size=n)
    x = p.linear_solve(b)
    Kd = K.toarray()
    be = np.max(np.abs(Kd @ x - b)) / (np.max(np.sum(np.abs(Kd), axis=1)) * np.max(np.abs(x)) + np.max(np.abs(b)))
    assert be <= 1e-14
    dy = p.linear_solve(step["rhs"])
    assert _close(dy, step["dy"], 1e-9)


def _cold_and_warm(m, p, ipm):
    """Cold solve on both sides, then one plant step (from the oracle's u_1, so
    both sides get the same new x0) and a warm re-solve of each side from its
    own previous (tightened) iterate."""
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    ref_t = solve_pair(m, p, ipm, ref, warm=False)
    x1 = m.step(m.x0, m.u1(ref_t.state.y))
    m.set_parameters(x0=x1)
    p.set_parameters(x1)
    ref2 = ipm.solve(ref_t.state, ipm.o.mu0_warm)
    assert ref2.status == 0
    solve_pair(m, p, ipm, ref2, warm=True)


@pytest.mark.parametrize("G,H,seed", [(8, 5, 1), (16, 10, 0)])
def test_plate_solve_matches_oracle(G, H, seed):
    _note(f"plate solve G={G} H={H} seed={seed}")
    w, m, p = _pair(G, H, seed)
    _cold_and_warm(m, p, LiftedIPM(m, _opts()))


@pytest.mark.parametrize("G,H", [(8, 3), (16, 10)])
def test_plate_adjoint_matches_oracle(G, H):
    """End to end: the GPU's sensitivities at its own cold solution (tightened
    on its barrier problem) against the oracle's at its own (1e-5).  Then the
    sensitivities at the oracle's point, placed on the GPU with set_iterate, at
    1e-6: 16 x 10 takes the large-front solves."""
    _note(f"plate adjoint G={G} H={H}")
    w, m, p = _pair(G, H)
    ipm = LiftedIPM(m, _opts())
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    ref = tighten_ref(ipm, ref)
    st = ref.state
    sens = sensitivities(ipm, st)
    rng = np.random.default_rng(4)
    su, so = rng.normal(size=16), float(rng.normal())
    r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL))
    assert r.status == 0
    tighten_gpu(p, r.mu)
    rc, J_own = p.jacobian_u1_x0()
    assert rc == 0
    rc, g_own = p.adjoint(su, so)
    assert rc == 0
    assert _close(J_own, sens["x0"]["du1"], 1e-5)
    for key in ("x0", "setpoint"):
        assert _close(g_own[key], su @ sens[key]["du1"] + so * sens[key]["df"], 1e-5), key
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "setpoint"):
        refg = su @ sens[key]["du1"] + so * sens[key]["df"]
        assert _close(g[key], refg, 1e-6), key
    assert np.all(g["u_prev"] == 0.0)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    assert _close(J, sens["x0"]["du1"], 1e-6)


def test_plate_full_size_sampled():
    """32 x 32 grid, horizon 50 (n = 52,000): the library's condensed matrix at
    a cold-start point equals the oracle's assembly entry by entry; the solve
    of it has a backward error at rounding level against the oracle's matrix;
    a cold solve converges and the oracle's evaluator certifies the
    optimality error of the original problem."""
    _note("plate full size G=32 H=50")
    w, m, p = _pair(32, 50)
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), 0.1)
    st.omega = np.random.default_rng(5).normal(scale=0.5, size=ipm.ml)
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    kv, rhs = p.assemble(0.1)
    lam = st.omega[:m.m_c] - st.omega[m.m_c:2 * m.m_c]
    W = m.hess(st.y, lam, np.zeros(0))
    gL, gU = ipm.gaps(st.y)
    sig = np.where(ipm.hasL, st.zL / gL, 0.0) + np.where(ipm.hasU, st.zU / gU, 0.0)
    Q = st.beta / st.s
    Jc = m.jac_c(st.y)
    K = (W + sp.diags(sig) + Jc.T @ sp.diags(Q[:m.m_c] + Q[m.m_c:]) @ Jc).tocsr()
    pat = p.patterns()
    ref = np.asarray(K[pat["k_rows"], pat["k_cols"]]).ravel()
    assert _close(kv, ref, 1e-12)
    eta = 0.0
    ok, _ = p.factor(kv, eta, want_l=False)
    while not ok:   # the random multipliers may make W indefinite: regularize as the method does
        eta = 1e-4 if eta == 0.0 else 100.0 * eta
        ok, _ = p.factor(kv, eta, want_l=False)
    K = (K + eta * sp.identity(m.n)).tocsr()
    x = p.linear_solve(rhs)
    be = np.max(np.abs(K @ x - rhs)) / (np.max(abs(K).sum(axis=1)) * np.max(np.abs(x)) + np.max(np.abs(rhs)))
    assert be <= 1e-13
    r = p.solve(warm=False)
    assert r.status == 0, r.status
    sol = p.solution()
    e = kkt_error(m, sol["y"], sol["lam"], np.zeros(0), sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
