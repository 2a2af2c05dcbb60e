"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Each step is checked on the same seeded inputs: model evaluation, condensed
assembly, supernodal Cholesky and solves, and whole interior-point solves of
NMPC episodes (solutions, multipliers, iteration counts, optimality error of
the original problem recomputed by the oracle's own evaluator).
"""
import sys

import numpy as np
import pytest

from paper_2606_04725_amd import nmpc as N
from oracle import symbolic as S
from oracle.distillation import DistillationOCP
from oracle.ipm import LiftedIPM
from oracle.kkt import kkt_error
from oracle.nmpc import distillation_episode
from workloads import distillation_workload

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _pair(Ntr, H, dt=0.1, alpha=2.5, seed=0):
    w = distillation_workload("small", seed, N=Ntr, H=H, dt=dt, alpha=alpha)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    p = N.Problem(N.distillation_structure(Ntr, H, dt, alpha))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    return w, m, p


def _rand_point(m, rng):
    y = rng.uniform(0.05, 0.95, m.n)
    for k in range(m.H):
        y[m.iR(k)] = rng.uniform(0.6, 4.5)
        y[m.iV(k)] = rng.uniform(0.6, 4.5)
    return y


def _close(a, b, tol):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(1.0, float(np.max(np.abs(b)))) if b.size else 1.0
    return float(np.max(np.abs(a - b))) / scale <= tol if b.size else True


@pytest.mark.parametrize("Ntr,H", [(10, 20), (40, 100), (2, 1)])
def test_eval_matches_oracle(Ntr, H):
    _note(f"eval N={Ntr} H={H}")
    w, m, p = _pair(Ntr, H)
    rng = np.random.default_rng(1)
    y = _rand_point(m, rng)
    lam = rng.normal(size=m.m_c)
    lam_d = rng.normal(size=m.m_d)
    out = p.eval(y, lam, lam_d)
    pat = p.patterns()
    assert abs(out["f"] - m.f(y)) <= 1e-13 * max(1.0, abs(m.f(y)))
    assert _close(out["grad"], m.grad(y), 1e-13)
    assert _close(out["c"], m.cons_c(y), 1e-13)
    assert _close(out["d"], m.cons_d(y), 1e-14)
    J = m.jac_c(y).tocsr()
    Jd = m.jac_d(y).tocsr()
    jr, jc = pat["j_rows"], pat["j_cols"]
    ref = np.array([J[r, c] if r < m.m_c else Jd[r - m.m_c, c] for r, c in zip(jr, jc)])
    assert _close(out["j_vals"], ref, 1e-13)
    W = m.hess(y, lam, lam_d).tocsr()
    refw = np.array([W[r, c] for r, c in zip(pat["w_rows"], pat["w_cols"])])
    assert _close(out["w_vals"], refw, 1e-13)


def _oracle_kkt_at_cold_start(m, mu=0.1, seed=0):
    ipm = LiftedIPM(m)
    st = ipm.cold_start(m.initial_guess(), mu)
    rng = np.random.default_rng(seed)
    st.omega = rng.normal(scale=0.5, size=ipm.ml)
    f, gf = m.f(st.y), m.grad(st.y)
    c, d = m.cons_c(st.y), m.cons_d(st.y)
    step = ipm.newton_step(st, mu, f, gf, c, d, m.jac_c(st.y), m.jac_d(st.y))
    return ipm, st, step


def _dense_L_from_panels(p, lv):
    sym = p.export_symbolic()
    n = p.n
    Ld = np.zeros((n, n))
    off = 0
    sp, rp, rows = sym["snode_ptr"], sym["snode_rows_ptr"], sym["snode_rows"]
    for s in range(sym["n_supernodes"]):
        f, l = sp[s], sp[s + 1]
        R = rows[rp[s]:rp[s + 1]]
        mr, w = len(R), l - f
        panel = lv[off:off + mr * w].reshape(w, mr).T
        off += mr * w
        upper = np.triu(panel[:w, :w], 1)
        assert np.all(upper == 0.0)
        for j in range(w):
            Ld[R[j:], f + j] = panel[j:, j]
    return Ld, sym


@pytest.mark.parametrize("Ntr,H", [(10, 20), (40, 100)])
def test_factor_and_solve_match_dense_cholesky(Ntr, H):
    _note(f"factor N={Ntr} H={H}")
    w, m, p = _pair(Ntr, H)
    ipm, st, step = _oracle_kkt_at_cold_start(m)
    K = step["K"].tocsr()
    pat = p.patterns()
    kv = np.asarray(K[pat["k_rows"], pat["k_cols"]]).ravel()
    eta = step["eta"]
    ok, lv = p.factor(kv, eta)
    assert ok
    Ld, sym = _dense_L_from_panels(p, lv)
    perm = sym["perm"]
    K = (K + eta * __import__("scipy.sparse", fromlist=["identity"]).identity(m.n)).tocsr()
    Kp = K.toarray()[np.ix_(perm, perm)]
    Lref = np.linalg.cholesky(Kp)
    assert np.linalg.norm(Ld - Lref) / np.linalg.norm(Lref) <= 1e-12
    # entries the exact factor does not have are stored as exact zeros
    r, c = S.kkt_lower_pattern(m)
    a = S.analyze(m.n, r, c, graph_stages=(m.H, m.ns, m.nx))
    mask = np.zeros((m.n, m.n), dtype=bool)
    for j, sset in enumerate(a["struct"]):
        mask[list(sset), j] = True
    assert np.all(Ld[~mask] == 0.0)
    # solve backward error
    rng = np.random.default_rng(2)
    b = rng.normal(size=m.n)
    x = p.linear_solve(b)
    Kd = K.toarray()
    be = np.max(np.abs(Kd @ x - b)) / (np.max(np.sum(np.abs(Kd), axis=1)) * np.max(np.abs(x)) + np.max(np.abs(b)))
    assert be <= 1e-14
    # the Newton direction of the oracle
    dy = p.linear_solve(step["rhs"])
    assert _close(dy, step["dy"], 1e-9)


def test_factor_detects_indefinite_and_regularizes():
    _note("factor indefinite")
    w, m, p = _pair(10, 20)
    ipm, st, step = _oracle_kkt_at_cold_start(m)
    K = step["K"].tocsr().toarray()
    j = m.n // 2
    K[j, j] = -abs(K[j, j]) - 1.0
    pat = p.patterns()
    kv = K[pat["k_rows"], pat["k_cols"]]
    ok, _ = p.factor(kv, 0.0, want_l=False)
    assert not ok
    lam_min = np.min(np.linalg.eigvalsh(K))
    ok2, _ = p.factor(kv, -lam_min + 1e-3, want_l=False)
    assert ok2
    kv_nan = kv.copy()
    kv_nan[0] = np.nan
    ok3, _ = p.factor(kv_nan, 0.0, want_l=False)
    assert not ok3


@pytest.mark.parametrize("mu", [1e-1, 1e-4])
def test_assemble_matches_oracle(mu):
    _note(f"assemble mu={mu}")
    w, m, p = _pair(10, 20)
    ipm, st, step = _oracle_kkt_at_cold_start(m, mu=0.1, seed=3)
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    step = ipm.newton_step(st, mu, m.f(st.y), m.grad(st.y), m.cons_c(st.y), m.cons_d(st.y), m.jac_c(st.y),
                           m.jac_d(st.y))
    kv, rhs = p.assemble(mu)
    pat = p.patterns()
    ref = np.asarray(step["K"].tocsr()[pat["k_rows"], pat["k_cols"]]).ravel()
    assert _close(kv, ref, 1e-12)
    assert _close(rhs, step["rhs"], 1e-12)


def _run_episode_gpu(w, recs):
    """Replay the oracle's parameter sequence on the GPU (warm start from the
    GPU's own previous solution)."""
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    out = []
    for i, rec in enumerate(recs):
        p.set_parameters(rec["x0"], setpoint=[w.xD_sp, w.xB_sp], traj=rec["zF"], u_prev=rec["u_prev"])
        r = p.solve(warm=i > 0)
        out.append((r, p.solution()))
    return out


def _compare_episode(w, m, recs, gpu, tol=1e-6):
    for rec, (r, sol) in zip(recs, gpu):
        assert r.status == 0, (rec["index"], r.status)
        m.set_parameters(x0=rec["x0"], zF=rec["zF"], u_prev=rec["u_prev"])
        e = kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])
        assert e["max"] <= 1e-8, (rec["index"], e)
        assert _close(sol["y"], rec["y"], tol), rec["index"]
        assert _close(sol["lam"], rec["lam"], tol), rec["index"]
        assert _close(sol["omega_d"], rec["omega_d"], tol), rec["index"]
        assert _close(sol["zL"], rec["zL"], tol) and _close(sol["zU"], rec["zU"], tol), rec["index"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ipm_episode_small_matches_oracle(seed):
    _note(f"episode small seed={seed}")
    w = distillation_workload("small", seed)
    m, recs = distillation_episode(w)
    gpu = _run_episode_gpu(w, recs)
    _compare_episode(w, m, recs, gpu)
    iters_o = [r["iters"] for r in recs]
    iters_g = [r.iters for r, _ in gpu]
    assert iters_g == iters_o


def test_ipm_episode_medium_matches_oracle():
    _note("episode medium seed=0 (cold + 3 warm)")
    w = distillation_workload("medium", 0)
    m, recs = distillation_episode(w, n_resolves=3)
    gpu = _run_episode_gpu(w, recs)
    _compare_episode(w, m, recs, gpu)


def test_single_stage_problem():
    _note("episode N=2 H=1")
    w = distillation_workload("small", 5, N=2, H=1, n_resolves=2)
    m, recs = distillation_episode(w)
    gpu = _run_episode_gpu(w, recs)
    _compare_episode(w, m, recs, gpu)


def test_solve_is_deterministic():
    _note("determinism")
    w, m, p = _pair(10, 20)
    p.solve()
    it0 = p.get_iterate()
    sols = []
    for _ in range(2):
        p.set_iterate(**it0)
        p.set_parameters(w.next_measurement(m.x1(it0["y"]), 0), setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(1),
                         u_prev=it0["y"][m.nx:m.nx + 2])
        r = p.solve(warm=True)
        sols.append((r.iters, p.get_iterate()))
    assert sols[0][0] == sols[1][0]
    for k in sols[0][1]:
        assert np.array_equal(sols[0][1][k], sols[1][1][k]), k
