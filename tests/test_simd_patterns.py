"""Index-data patterns of the stage-pattern front end (eq. 3: one pattern
repeated over discretization points), on the CPU: the workload plate written
as one stencil row pattern and one tracking pattern, its per-stage structure
and its values, Jacobian, Lagrangian Hessian, gradient and objective
(emulating the generated kernels' scratch positions and summation lists)
against the oracle's own transcription of the plate (oracle/plate.py), and
the generator's rules."""
import numpy as np
import pytest

from oracle.plate import PlateOCP
from paper_2606_04725_amd import simd_models as SM
from paper_2606_04725_amd import simd_patterns as SPn
from paper_2606_04725_amd.simd import sin
from simd_eval import expand_patterns


def _pair(G=8, H=3, dt=0.01, seed=0):
    m = PlateOCP(G, H, dt)
    rng = np.random.default_rng(seed)
    m.set_parameters(x0=rng.uniform(0.0, 1.2, m.nx), target=rng.uniform(0.2, 1.0, m.nx))
    g = SPn.generate(SM.plate_pattern_model(G))
    return m, g, rng


@pytest.mark.parametrize("G", [4, 8])
def test_plate_pattern_structure_matches_the_oracle(G):
    m, g, rng = _pair(G)
    assert (g.nx, g.nu, g.n_setpoint) == (m.nx, m.nu, m.nx)
    y = rng.uniform(0.0, 1.2, m.n)
    out = expand_patterns(g, y, m.H, m.x0, m.dt, m.target, lam=rng.normal(size=m.m_c))
    J = m.jac_c(y).tocsr()
    got = set(zip(out["jr"].tolist(), out["jc"].tolist()))
    assert len(got) == len(out["jr"])
    assert got == set(zip(*J.nonzero()))
    W = m.hess(y, rng.normal(size=m.m_c), np.zeros(0)).tocsr()
    Wl = set((a, b) for a, b in zip(*W.nonzero()) if a >= b)
    assert Wl <= set(zip(out["wr"].tolist(), out["wc"].tolist()))
    lo, hi = np.tile(g.lb, m.H), np.tile(g.ub, m.H)
    assert np.array_equal(lo, m.lb) and np.array_equal(hi, m.ub)


@pytest.mark.parametrize("G,seed", [(4, 1), (8, 2)])
def test_plate_pattern_values_match_the_oracle(G, seed):
    m, g, rng = _pair(G, seed=seed)
    y = rng.uniform(0.0, 1.2, m.n)
    lam = rng.normal(size=m.m_c)
    out = expand_patterns(g, y, m.H, m.x0, m.dt, m.target, lam=lam)
    assert abs(out["f"] - m.f(y)) <= 1e-13 * abs(m.f(y))
    assert np.max(np.abs(out["grad"] - m.grad(y))) <= 1e-13 * np.max(np.abs(m.grad(y)))
    assert np.max(np.abs(out["c"] - m.cons_c(y))) <= 1e-12 * np.max(np.abs(m.cons_c(y)))
    J = m.jac_c(y).tocsr()
    want = np.asarray(J[out["jr"], out["jc"]]).ravel()
    assert not np.isnan(out["jv"]).any()
    assert np.max(np.abs(out["jv"] - want)) <= 1e-13 * np.max(np.abs(want))
    W = m.hess(y, lam, np.zeros(0)).tocsr()
    want = np.asarray(W[out["wr"], out["wc"]]).ravel()
    assert np.max(np.abs(out["wv"] - want)) <= 1e-12 * np.max(np.abs(want))


def test_scratch_lists_partition_the_scratch():
    """Every scratch double a kernel writes is summed exactly once."""
    g = SPn.generate(SM.plate_pattern_model(8))
    _, st = g.pattern_structure
    seen = [q for lists in ("w_lists", "g_lists", "f_lists") for l in st[lists] for q in l]
    assert sorted(seen) == list(range(st["ncoo"]))
    assert g.scratch_per_stage == st["ncoo"] == 8 * 8 * 5 + 8 * 8 * 3
    assert "nmpc_stage_reduce" in g.source and "nmpc_stage_eval" in g.source


def test_pattern_with_data_and_setpoints():
    """Two row patterns with per-instance data and an objective with two
    setpoint slots and the stage trajectory, against direct evaluation."""
    m = SPn.PatternModel("mixed", n_setpoint=3)
    X = m.states(4, lb=-5.0)
    U = m.controls(2, lb=-1.0, ub=1.0)
    tr = m.traj()
    m.row_pattern(lambda v, p, d: v[0] - p[0] - m.dt * (d[0] * v[1] + d[1] * sin(v[0])),
                  [dict(target=X[0], vars=[X[0], U[0]], prevs=[X[0]], data=[1.5, 0.3]),
                   dict(target=X[1], vars=[X[1], U[1]], prevs=[X[1]], data=[-0.5, 0.7])], nv=2, nprev=1, ndata=2)
    m.row_pattern(lambda v, p, d: 2.0 * v[0] - p[0] + 0.5 * p[1] - v[1] * v[1],
                  [dict(target=X[2], vars=[X[2], X[0]], prevs=[X[2], X[3]]),
                   dict(target=X[3], vars=[X[3], X[1]], prevs=[X[3], X[0]])], nv=2, nprev=2)
    m.objective_pattern(lambda v, d, s: d[0] * (v[0] - s[0]) ** 2 + (v[1] - s[1] * tr) ** 2,
                        [dict(vars=[X[0], U[0]], data=[2.0], sps=[0, 2]),
                         dict(vars=[X[3], U[1]], data=[0.5], sps=[1, 2])], nv=2, ndata=1, nsp=2)
    g = SPn.generate(m)
    assert g.uses_traj
    H, dt = 3, 0.1
    rng = np.random.default_rng(5)
    y, x0, sp, traj = rng.normal(size=H * 6), rng.normal(size=4), rng.normal(size=3), rng.normal(size=H)
    lam = rng.normal(size=H * 4)
    out = expand_patterns(g, y, H, x0, dt, sp, traj, lam)

    def rows(y):
        Y = y.reshape(H, 6)
        P = np.vstack([x0, Y[:-1, :4]])
        r = np.empty((H, 4), dtype=y.dtype)
        r[:, 0] = Y[:, 0] - P[:, 0] - dt * (1.5 * Y[:, 4] + 0.3 * np.sin(Y[:, 0]))
        r[:, 1] = Y[:, 1] - P[:, 1] - dt * (-0.5 * Y[:, 5] + 0.7 * np.sin(Y[:, 1]))
        r[:, 2] = 2.0 * Y[:, 2] - P[:, 2] + 0.5 * P[:, 3] - Y[:, 0] ** 2
        r[:, 3] = 2.0 * Y[:, 3] - P[:, 3] + 0.5 * P[:, 0] - Y[:, 1] ** 2
        return r.reshape(-1)

    def obj(y):
        Y = y.reshape(H, 6)
        return np.sum(2.0 * (Y[:, 0] - sp[0]) ** 2 + (Y[:, 4] - sp[2] * traj) ** 2
                      + 0.5 * (Y[:, 3] - sp[1]) ** 2 + (Y[:, 5] - sp[2] * traj) ** 2)

    assert np.max(np.abs(out["c"] - rows(y))) <= 1e-14
    assert abs(out["f"] - obj(y)) <= 1e-12
    hcs = 1e-30
    E = np.eye(H * 6)
    Jcs = np.array([rows(y + 1j * hcs * E[i]).imag / hcs for i in range(H * 6)]).T
    assert np.max(np.abs(out["jv"] - Jcs[out["jr"], out["jc"]])) <= 1e-14
    assert np.count_nonzero(Jcs) == len(out["jv"])
    gcs = np.array([obj(y + 1j * hcs * E[i]).imag / hcs for i in range(H * 6)])
    assert np.max(np.abs(out["grad"] - gcs)) <= 1e-13

    def lag_grad(y):
        return np.array([(obj(y + 1j * hcs * E[i]) + lam @ rows(y + 1j * hcs * E[i])).imag / hcs
                         for i in range(H * 6)])

    h = 1e-6
    Wfd = np.array([(lag_grad(y + h * E[i]) - lag_grad(y - h * E[i])) / (2 * h) for i in range(H * 6)])
    assert np.max(np.abs(out["wv"] - Wfd[out["wr"], out["wc"]])) <= 1e-7
    on = set(zip(out["wr"].tolist(), out["wc"].tolist()))
    assert all((a, b) in on for a, b in zip(*np.nonzero(np.abs(np.tril(Wfd)) > 1e-6)))


def test_generator_rules():
    def model():
        m = SPn.PatternModel("bad")
        X = m.states(2)
        U = m.controls(1)
        return m, X, U

    m, X, U = model()
    m.row_pattern(lambda v, p, d: v[0] - p[0] - v[1], [dict(target=X[0], vars=[X[0], U[0]], prevs=[X[0]])],
                  nv=2, nprev=1)
    with pytest.raises(ValueError, match="without a row"):
        SPn.generate(m)
    m, X, U = model()
    inst = [dict(target=X[0], vars=[X[1], U[0]], prevs=[X[0]]), dict(target=X[1], vars=[X[1], U[0]], prevs=[X[1]])]
    m.row_pattern(lambda v, p, d: v[0] - p[0] - v[1], inst, nv=2, nprev=1)
    with pytest.raises(ValueError, match="own state"):
        SPn.generate(m)
    m, X, U = model()
    inst = [dict(target=X[0], vars=[X[0], X[0]], prevs=[X[0]]), dict(target=X[1], vars=[X[1], U[0]], prevs=[X[1]])]
    m.row_pattern(lambda v, p, d: v[0] - p[0] - v[1], inst, nv=2, nprev=1)
    with pytest.raises(ValueError, match="distinct"):
        SPn.generate(m)
    m, X, U = model()
    inst = [dict(target=X[j], vars=[X[j], U[0]], prevs=[X[j]]) for j in range(2)]
    m.row_pattern(lambda v, p, d: v[0] - p[0] * p[0] - v[1], inst, nv=2, nprev=1)
    with pytest.raises(ValueError, match="linearly"):
        SPn.generate(m)
    m, X, U = model()
    m.row_pattern(lambda v, p, d: v[0] - p[0] - v[1], [dict(target=X[j], vars=[X[j], U[0]], prevs=[X[j]])
                                                        for j in range(2)], nv=2, nprev=1)
    m.objective_pattern(lambda v, d, s: (v[0] - s[0]) ** 2, [dict(vars=[X[0]], sps=[3])], nv=1, nsp=1)
    with pytest.raises(ValueError, match="setpoint"):
        SPn.generate(m)
    m, X, U = model()
    with pytest.raises(ValueError, match="before the controls"):
        m.states(1)


def _stage_symbolic_case(kind):
    from oracle.distillation import DistillationOCP
    from oracle.plate_case import PlateCaseOCP
    from paper_2606_04725_amd import simd
    if kind == "plate8":
        return simd.compile(SM.plate_pattern_model(8)), PlateOCP(8, 6, 0.01)
    if kind == "plate16":
        return simd.compile(SM.plate_pattern_model(16)), PlateOCP(16, 10, 0.01)
    if kind == "column":
        return (simd.compile(SM.distillation_model(6, 2.3, F=1.0, rho=0.05)),
                DistillationOCP(6, 30, 0.1, 2.3, F=1.0, rho=0.05))
    return simd.compile(SM.plate_case_model(n=9)), PlateCaseOCP(H=5, n=9)


@pytest.mark.parametrize("kind", ["plate8", "plate16", "column", "plate_case"])
def test_stage_model_symbolic_bit_exact_vs_oracle(kind):
    """The library's analysis of a front-end model (its default ordering, the
    stage-and-graph nested dissection, told only the patterns and the number
    of states) equals the oracle's on the oracle model's own condensed
    pattern: permutation, elimination tree, column counts and supernodes."""
    from oracle import symbolic as S
    from paper_2606_04725_amd import nmpc as N
    g, m = _stage_symbolic_case(kind)
    p = N.Problem(N.stage_model_structure(g, m.H, m.dt))
    p.analyze()
    lib = p.export_symbolic()
    r, c = S.kkt_lower_pattern(m)
    pat = p.patterns()
    assert set(zip(pat["k_rows"].tolist(), pat["k_cols"].tolist())) == set(zip(r, c))
    a = S.analyze(m.n, r, c, graph_stages=(m.H, m.ns, m.nx))
    assert np.array_equal(lib["perm"], a["perm"])
    assert np.array_equal(lib["parent"], a["parent"])
    assert np.array_equal(lib["colcount"], a["colcount"])
    assert np.array_equal(lib["snode_ptr"], a["snode_ptr"])
    rp = lib["snode_rows_ptr"]
    for s_, rows in enumerate(a["snode_rows"]):
        assert np.array_equal(lib["snode_rows"][rp[s_]:rp[s_ + 1]], rows)
    assert lib["nnz_l"] == a["nnz_L"] and lib["flops"] == a["flops"]
    p.close()


@pytest.mark.parametrize("n,seed", [(9, 3), (21, 4)])
def test_case_study_plate_as_patterns_matches_the_oracle(n, seed):
    """The heated-plate case study (Section 4.2) written as six row patterns
    and two objective patterns: values and derivatives against the oracle's
    transcription (oracle/plate_case.py)."""
    from oracle.plate_case import PlateCaseOCP
    m = PlateCaseOCP(H=3, n=n)
    rng = np.random.default_rng(seed)
    m.set_parameters(x0=rng.uniform(40.0, 70.0, m.nx), traj=rng.uniform(54.0, 64.0, m.H))
    g = SPn.generate(SM.plate_case_pattern_model(n=n))
    assert (g.nx, g.nu) == (m.nx, 1)
    y = rng.uniform(40.0, 70.0, m.n)
    y[m.nx::m.ns] = rng.uniform(0.2, 2.0, m.H)
    lam = rng.normal(size=m.m_c)
    out = expand_patterns(g, y, m.H, m.x0, m.dt, (), m.traj, lam=lam)
    assert abs(out["f"] - m.f(y)) <= 1e-13 * abs(m.f(y))
    assert np.max(np.abs(out["grad"] - m.grad(y))) <= 1e-13 * np.max(np.abs(m.grad(y)))
    assert np.max(np.abs(out["c"] - m.cons_c(y))) <= 1e-12 * max(1.0, np.max(np.abs(m.cons_c(y))))
    J = m.jac_c(y).tocsr()
    want = np.asarray(J[out["jr"], out["jc"]]).ravel()
    assert set(zip(out["jr"].tolist(), out["jc"].tolist())) == set(zip(*J.nonzero()))
    assert np.max(np.abs(out["jv"] - want)) <= 1e-13 * np.max(np.abs(want))
    W = m.hess(y, lam, np.zeros(0)).tocsr()
    want = np.asarray(W[out["wr"], out["wc"]]).ravel()
    assert np.max(np.abs(out["wv"] - want)) <= 1e-12 * np.max(np.abs(want))
    lo = np.tile(g.lb, m.H)
    assert np.array_equal(np.isfinite(lo), np.isfinite(m.lb)) and np.allclose(lo[np.isfinite(lo)], m.lb[np.isfinite(m.lb)])


def test_case_study_column_as_patterns_matches_the_oracle():
    """The distillation case study (Section 4.1) written with tray, feed,
    condenser and reboiler row patterns, algebraic equilibrium and flow
    patterns and guess patterns: values, derivatives and the cold-start guess
    against the oracle's transcription (oracle/reflux.py)."""
    from oracle.reflux import RefluxColumnOCP
    from workloads import reflux_workload
    w = reflux_workload(H=4)
    m = RefluxColumnOCP(H=4)
    rng = np.random.default_rng(7)
    x0 = rng.uniform(0.1, 0.9, m.N)
    m.set_parameters(x0=x0, setpoint=[w.xbar, w.ubar], u_prev=[2.3])
    g = SPn.generate(SM.reflux_pattern_model(N=w.N, Nf=w.Nf, D=w.D, F=w.F, alpha=w.alpha, xf=w.xf, Ac=w.Ac,
                                              At=w.At, Ar=w.Ar, w_u=w.w_u))
    assert (g.nx, g.nu, g.na, g.n_alg_rows) == (m.N, 1, m.N + 3, m.N + 3)
    y = m.initial_guess() + rng.normal(scale=0.05, size=m.n)
    lam = rng.normal(size=m.m_c)
    out = expand_patterns(g, y, m.H, x0, m.dt, [w.xbar, w.ubar], lam=lam, u_prev=[2.3])
    assert np.max(np.abs(out["guess"] - m.initial_guess())) <= 1e-15
    assert abs(out["f"] - m.f(y)) <= 1e-14 * max(1.0, abs(m.f(y)))
    assert np.max(np.abs(out["grad"] - m.grad(y))) <= 1e-14
    assert np.max(np.abs(out["c"] - m.cons_c(y))) <= 1e-13
    J = m.jac_c(y).tocsr()
    assert set(zip(out["jr"].tolist(), out["jc"].tolist())) == set(zip(*J.nonzero()))
    want = np.asarray(J[out["jr"], out["jc"]]).ravel()
    assert np.max(np.abs(out["jv"] - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))
    W = m.hess(y, lam, np.zeros(0)).tocsr()
    want = np.asarray(W[out["wr"], out["wc"]]).ravel()
    assert np.max(np.abs(out["wv"] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))


def test_inequality_patterns_against_direct_evaluation():
    """Inequality rows from a pattern (one per instance), with an algebraic
    variable and a guess pattern: values, Jacobian rows after the equality
    rows, Hessian weighted by the inequality multipliers."""
    m = SM.row_kinds_model()
    g = SPn.generate(m)
    assert (g.na, g.n_alg_rows, len(g.ineq_ptr) - 1) == (1, 1, 2)
    H, dt = 3, 0.2
    rng = np.random.default_rng(9)
    y, x0 = rng.normal(size=H * 5), rng.normal(size=2)
    lam, lam_d = rng.normal(size=H * 3), rng.uniform(0.1, 1.0, size=H * 2)
    out = expand_patterns(g, y, H, x0, dt, lam=lam, lam_d=lam_d, u_prev=[0.3, -0.2])
    Y = y.reshape(H, 5)
    dd = np.stack([2.0 * Y[:, 2] ** 2 + Y[:, 1] - 1.0, 0.5 * Y[:, 3] ** 2 + Y[:, 4] - 3.0], axis=1).reshape(-1)
    assert np.max(np.abs(out["d"] - dd)) <= 1e-14
    mc = H * 3
    assert set(out["jr"][out["jr"] >= mc].tolist()) == set(range(mc, mc + H * 2))
    assert np.allclose(out["guess"][4::5], x0[0] * x0[1] + 0.25)
    # Hessian of lam^T c + lam_d^T d + f against central differences of its gradient
    hcs = 1e-30
    E = np.eye(H * 5)

    def lagr(yy):
        Yy = yy.reshape(H, 5)
        P = np.vstack([x0, Yy[:-1, :2]])
        c = np.stack([Yy[:, 0] - P[:, 0] - dt * Yy[:, 2] ** 2, Yy[:, 1] - P[:, 1] - dt * Yy[:, 3] ** 2,
                      Yy[:, 4] - Yy[:, 0] * Yy[:, 1]], axis=1).reshape(-1)
        d = np.stack([2.0 * Yy[:, 2] ** 2 + Yy[:, 1] - 1.0, 0.5 * Yy[:, 3] ** 2 + Yy[:, 4] - 3.0],
                     axis=1).reshape(-1)
        f = np.sum((Yy[:, 0] - 1.0) ** 2 + Yy[:, 4] ** 2)
        return f + lam @ c + lam_d @ d

    def grad(yy):
        return np.array([lagr(yy + 1j * hcs * E[i]).imag / hcs for i in range(H * 5)])

    h = 1e-6
    Wfd = np.array([(grad(y + h * E[i]) - grad(y - h * E[i])) / (2 * h) for i in range(H * 5)])
    assert np.max(np.abs(out["wv"] - Wfd[out["wr"], out["wc"]])) <= 1e-7


@pytest.mark.parametrize("N_,H", [(6, 4), (10, 3)])
def test_workload_column_as_patterns_matches_the_oracle(N_, H):
    """The workload column written as patterns (the feed tray reads the
    stage's feed composition; the move penalty reads the previous stage's
    controls, whose gradient and Hessian terms are summed into the previous
    stage and whose cross terms fill the cross-stage slots): values and
    derivatives against the oracle's column (oracle/distillation.py), and
    exactly its KKT pattern."""
    from oracle.distillation import DistillationOCP
    from oracle import symbolic as S
    m = DistillationOCP(N_, H, 0.1, 2.3, F=1.0, rho=0.05)
    rng = np.random.default_rng(N_)
    zF = rng.uniform(0.4, 0.6, H)
    up = rng.uniform(1.0, 3.0, 2)
    m.set_parameters(x0=rng.uniform(0.05, 0.95, m.nx), zF=zF, u_prev=up)
    g = SPn.generate(SM.distillation_pattern_model(N_, 2.3, F=1.0, rho=0.05))
    y = m.initial_guess() + rng.normal(scale=0.05, size=m.n)
    lam, lam_d = rng.normal(size=m.m_c), rng.uniform(0.1, 1.0, m.m_d)
    sp = [m.xD_sp, m.xB_sp]
    out = expand_patterns(g, y, H, m.x0, m.dt, sp, zF, lam=lam, lam_d=lam_d, u_prev=up)
    assert abs(out["f"] - m.f(y)) <= 1e-14 * max(1.0, abs(m.f(y)))
    assert np.max(np.abs(out["grad"] - m.grad(y))) <= 1e-13
    assert np.max(np.abs(out["c"] - m.cons_c(y))) <= 1e-13
    assert np.max(np.abs(out["d"] - m.cons_d(y))) <= 1e-14
    Jc, Jd = m.jac_c(y).tocsr(), m.jac_d(y).tocsr()
    import scipy.sparse as sps
    J = sps.vstack([Jc, Jd]).tocsr()
    assert set(zip(out["jr"].tolist(), out["jc"].tolist())) == set(zip(*J.nonzero()))
    want = np.asarray(J[out["jr"], out["jc"]]).ravel()
    assert np.max(np.abs(out["jv"] - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))
    W = m.hess(y, lam, lam_d).tocsr()
    want = np.asarray(W[out["wr"], out["wc"]]).ravel()
    assert np.max(np.abs(out["wv"] - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
    Wl = set((a, b) for a, b in zip(*W.nonzero()) if a >= b)
    assert Wl <= set(zip(out["wr"].tolist(), out["wc"].tolist()))


def test_generation_is_deterministic_and_tagged_by_content():
    """The same pattern model generates the same source and tag (the code
    object cache relies on it); a change of one instance's data changes both."""
    a = SPn.generate(SM.plate_case_pattern_model(n=9))
    b = SPn.generate(SM.plate_case_pattern_model(n=9))
    assert a.source == b.source and a.tag == b.tag
    c = SPn.generate(SM.plate_case_pattern_model(n=9, Tb=51.0))
    assert c.tag != a.tag and c.source != a.source
    assert f"TAG = {a.tag}ULL" in a.source
