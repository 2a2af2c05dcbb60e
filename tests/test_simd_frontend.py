"""Stage-pattern front end (eq. 3) on the CPU.

The expressions the front end derives once per pattern (rows, Jacobian,
gradient, Hessian of the Lagrangian, cold-start guess, parameter
contractions) are evaluated on the host and compared with the oracle's own
model functions, which are pinned by complex step elsewhere: the toy problem of
the re-solve listing (Section 3.3), a linear-quadratic problem (dynamics
through a constant matrix), the distillation case study of Section 4.1 with
its algebraic variables, the workload column (inequality rows, move
penalty on the previous stage's controls) and the heated-plate case study of
Section 4.2 (a 5-point stencil over the grid, nonlinear heated edges).  Then: the patterns cover every
nonzero, the C ABI takes the descriptor and rejects malformed ones, and the
two columns get the same KKT pattern and symbolic analysis as the library's
hand-written REFLUX_COLUMN and DISTILLATION families."""
import ctypes as C

import numpy as np
import pytest

from oracle.lq import LQOCP
from oracle.reflux import RefluxColumnOCP
from oracle.toy import ToyOCP
from paper_2606_04725_amd import capi, simd
from paper_2606_04725_amd import nmpc as N
from paper_2606_04725_amd import simd_models as SM
from simd_eval import contraction, ev, expand
from workloads import random_lq

TOL = 1e-12


def _toy():
    m = ToyOCP()
    traj = np.sin(m.t + 0.4)
    m.set_parameters(y0=0.7, traj=traj)
    return dict(name="toy", gm=SM.toy_model(), om=m, H=m.H, dt=m.dt, x0=np.array([0.7]), sp=(), traj=traj,
                up=np.array([0.0]), sp_group=None, tr_group="traj")


def _lq():
    A, B, Q, R, x0, xs = random_lq(4, 2, 20, seed=0)
    m = LQOCP(A, B, Q, R, 20, xs=xs)
    m.set_parameters(x0=x0)
    return dict(name="lq", gm=SM.lq_model(A, B, Q, R), om=m, H=20, dt=1.0, x0=x0, sp=xs, traj=None,
                up=np.zeros(2), sp_group="xs", tr_group=None)


def _distillation():
    from oracle.distillation import DistillationOCP
    m = DistillationOCP(6, 5, 0.1, 2.3, F=1.0, rho=0.05)
    rng = np.random.default_rng(1)
    m.set_parameters(x0=rng.uniform(0.1, 0.9, m.nx), zF=rng.uniform(0.4, 0.6, m.H), u_prev=[1.5, 2.2],
                     setpoint=[0.93, 0.07])
    gm = SM.distillation_model(6, 2.3, F=1.0, rho=0.05)
    return dict(name="distillation", gm=gm, om=m, H=5, dt=0.1, x0=m.x0, sp=np.array([0.93, 0.07]), traj=m.zF,
                up=m.u_prev, sp_group="setpoint", tr_group="zF", up_group="u_prev")


def _reflux():
    m = RefluxColumnOCP(5, N=8, Nf=4, w_u=0.3)
    m.set_parameters(setpoint=[0.9, 2.4], u_prev=[2.2])
    gm = SM.reflux_model(N=8, Nf=4, w_u=0.3)
    return dict(name="reflux", gm=gm, om=m, H=5, dt=m.dt, x0=m.x0, sp=np.array([0.9, 2.4]), traj=None,
                up=np.array([2.2]), sp_group="setpoint", tr_group=None)


def _plate_case():
    from oracle.plate_case import PlateCaseOCP
    m = PlateCaseOCP(H=3, n=9)
    rng = np.random.default_rng(2)
    m.set_parameters(x0=rng.uniform(40.0, 70.0, m.nx), traj=[58.0, 55.0, 63.0], u_prev=[0.6])
    return dict(name="plate_case", gm=SM.plate_case_model(n=9), om=m, H=3, dt=m.dt, x0=m.x0, sp=(), traj=m.traj,
                up=m.u_prev, sp_group=None, tr_group="traj")


CASES = {"toy": _toy, "lq": _lq, "reflux": _reflux, "distillation": _distillation, "plate_case": _plate_case}


def _point(c, rng):
    om = c["om"]
    y = rng.uniform(0.1, 0.9, om.n)
    if c["name"] == "reflux":
        Y = y.reshape(om.H, om.ns)
        Y[:, om.iu] = rng.uniform(1.5, 3.0, om.H)
        Y[:, om.iL:] = rng.uniform(0.3, 1.5, (om.H, 3))
    return y


@pytest.mark.parametrize("case", list(CASES))
def test_generated_expressions_equal_the_oracle_model(case):
    c = CASES[case]()
    d = simd.derive(c["gm"])
    om = c["om"]
    rng = np.random.default_rng(4)
    y = _point(c, rng)
    lam, lam_d = rng.normal(size=om.m_c), rng.normal(size=om.m_d)
    e = expand(d, y, c["H"], c["x0"], c["dt"], c["sp"], c["traj"], lam, lam_d, c["up"])
    scale = lambda v: max(1.0, float(np.max(np.abs(v))))
    assert abs(e["f"] - om.f(y)) <= TOL * scale(om.f(y))
    assert np.max(np.abs(e["grad"] - om.grad(y))) <= TOL * scale(om.grad(y))
    assert np.max(np.abs(e["c"] - om.cons_c(y))) <= TOL * scale(om.cons_c(y))
    if om.m_d:
        assert np.max(np.abs(e["d"] - om.cons_d(y))) <= TOL * scale(om.cons_d(y))
        J = np.vstack([om.jac_c(y).toarray(), om.jac_d(y).toarray()])
    else:
        J = om.jac_c(y).toarray()
    assert np.max(np.abs(e["jv"] - J[e["jr"], e["jc"]])) <= TOL * scale(J)
    mask = np.zeros_like(J, dtype=bool)
    mask[e["jr"], e["jc"]] = True
    assert np.all(J[~mask] == 0.0), "the oracle's Jacobian has an entry outside the generated pattern"
    W = om.hess(y, lam, lam_d).toarray()
    assert np.max(np.abs(e["wv"] - W[e["wr"], e["wc"]])) <= TOL * scale(W)
    wmask = np.zeros_like(W, dtype=bool)
    wmask[e["wr"], e["wc"]] = True
    low = np.tril(np.ones_like(W, dtype=bool))
    assert np.all(W[low & ~wmask] == 0.0), "the oracle's Hessian has an entry outside the generated pattern"
    # rows are ordered previous-stage columns first, then own columns: ascending
    for r in range(om.m_c + om.m_d):
        cols = e["jc"][e["jr"] == r]
        assert np.all(np.diff(cols) > 0)


@pytest.mark.parametrize("case", list(CASES))
def test_generated_guess_equals_the_oracle_cold_start(case):
    c = CASES[case]()
    d = simd.derive(c["gm"])
    env = {("dt", 0): c["dt"]}
    for i, v in enumerate(c["x0"]):
        env[("x0", i)] = v
    for j, v in enumerate(c["up"]):
        env[("up", j)] = v
    for j, v in enumerate(c["sp"]):
        env[("sp", j)] = v
    g = np.array([[ev(d.guess[j], {**env, ("tr", 0): 0.0 if c["traj"] is None else c["traj"][k]})
                   for j in range(d.model.ns)] for k in range(c["H"])]).reshape(-1)
    want = c["om"].initial_guess()
    assert np.max(np.abs(g - want)) <= 1e-15


@pytest.mark.parametrize("case", list(CASES))
def test_parameter_contractions_equal_differences_of_the_oracle(case):
    """The adjoint kernel's contraction for a parameter p,
    -w . d(grad_y L)/dp - al . dc/dp + so df/dp, against central differences
    of the same quantity built from the oracle's functions (the parameters
    enter at most quadratically, so the differences are exact to rounding)."""
    c = CASES[case]()
    d = simd.derive(c["gm"])
    om = c["om"]
    rng = np.random.default_rng(9)
    y = _point(c, rng)
    lam, lam_d = rng.normal(size=om.m_c), rng.normal(size=om.m_d)
    al, w, so = rng.normal(size=om.m_c + om.m_d), rng.normal(size=om.n), 0.7
    gsp, gtr, gup = contraction(d, y, c["H"], c["x0"], c["dt"], c["sp"], c["traj"], lam, al, w, so, lam_d,
                                c["up"])

    def phi():
        gl = om.grad(y) + om.jac_c(y).T @ lam
        val = -w @ gl - al[:om.m_c] @ om.cons_c(y) + so * om.f(y)
        if om.m_d:
            val += -w @ (om.jac_d(y).T @ lam_d) - al[om.m_c:] @ om.cons_d(y)
        return val

    def fd(setter, base, idx, h=1e-4):
        vals = []
        for sgn in (1, -1):
            v = np.array(base, dtype=float).copy()
            v[idx] += sgn * h
            setter(v)
            vals.append(phi())
        setter(np.array(base, dtype=float))
        return (vals[0] - vals[1]) / (2 * h)

    if c["sp_group"]:
        g = c["sp_group"]
        for j in range(len(c["sp"])):
            want = fd(lambda v: om.set_parameters(**{g: v}), c["sp"], j)
            assert abs(gsp[j] - want) <= 1e-8 * max(1.0, abs(want)), (j, gsp[j], want)
    else:
        assert gsp.size == 0
    if c["tr_group"]:
        g = c["tr_group"]
        for k in sorted({0, min(3, c["H"] - 1), c["H"] - 1}):
            want = fd(lambda v: om.set_parameters(**{g: v}), c["traj"], k)
            assert abs(gtr[k] - want) <= 1e-8 * max(1.0, abs(want)), (k, gtr[k], want)
    if c.get("up_group"):
        g = c["up_group"]
        for b in range(len(c["up"])):
            want = fd(lambda v: om.set_parameters(**{g: v}), c["up"], b)
            assert abs(gup[b] - want) <= 1e-8 * max(1.0, abs(want)), (b, gup[b], want)
    else:
        assert np.all(gup == 0.0)


def test_model_validation():
    m = simd.StageModel("bad_obj")
    x = m.state("x")
    u = m.control("u")
    m.dynamics(x, u)
    m.minimize(m.prev(x) ** 2)
    with pytest.raises(ValueError):
        simd.derive(m)
    m = simd.StageModel("nonlinear_prev")
    x = m.state("x")
    u = m.control("u")
    m.state_equation(x, x - m.prev(x) ** 2 - u)
    with pytest.raises(ValueError):
        simd.derive(m)
    m = simd.StageModel("no_equation")
    x = m.state("x")
    m.state("z")
    m.control("u")
    m.dynamics(x, x)
    with pytest.raises(ValueError):
        simd.derive(m)
    m = simd.StageModel("bad_guess")
    x = m.state("x")
    u = m.control("u")
    m.dynamics(x, u)
    m.guess(u, x)
    with pytest.raises(ValueError):
        simd.derive(m)
    m = simd.StageModel("alg_prev")
    x = m.state("x")
    u = m.control("u")
    m.dynamics(x, u)
    m.equality(u - m.prev(x))
    with pytest.raises(ValueError):
        simd.derive(m)


def test_inequality_and_previous_control_validation():
    m = simd.StageModel("ineq_prev")
    x = m.state("x")
    u = m.control("u")
    m.dynamics(x, u)
    m.inequality(u - m.prev(x))
    with pytest.raises(ValueError):
        simd.derive(m)
    m = simd.StageModel("rows_prev_control")
    x = m.state("x")
    u = m.control("u")
    m.dynamics(x, u - m.prev_control(u))
    with pytest.raises(ValueError):
        simd.derive(m)


@pytest.fixture(scope="module")
def compiled():
    return {k: simd.compile(CASES[k]()["gm"]) for k in CASES}


def test_compile_produces_a_code_object(compiled):
    for g in compiled.values():
        assert len(g.code) > 1000 and g.tag != 0
        with open(g.path, "rb") as fh:
            assert fh.read() == g.code


def test_case_study_model_gets_the_hand_written_pattern(compiled):
    """The front end's case-study column and the REFLUX_COLUMN family
    transcribe the same problem: same sizes, Jacobian and Hessian patterns
    (as sets) and the same symbolic analysis."""
    H = 6
    pg = N.Problem(N.stage_model_structure(compiled["reflux"], H, 2.0))
    ph = N.Problem(N.reflux_structure(H, N=8, Nf=4, w_u=0.3))
    assert (pg.n, pg.m_c, pg.m_d, pg.nx, pg.nu, pg.nnz_k) == (ph.n, ph.m_c, ph.m_d, ph.nx, ph.nu, ph.nnz_k)
    pg.analyze()
    ph.analyze()
    a, b = pg.patterns(), ph.patterns()
    for rk, ck in (("j_rows", "j_cols"), ("w_rows", "w_cols")):
        sa = set(zip(a[rk].tolist(), a[ck].tolist()))
        sb = set(zip(b[rk].tolist(), b[ck].tolist()))
        assert sa == sb, rk
    assert pg.symbolic_sizes() == ph.symbolic_sizes()
    assert pg.n_setpoint == 2 and pg.n_traj == 0


def test_workload_column_model_gets_the_hand_written_pattern(compiled):
    """The front end's workload column (inequality rows, move penalty on the
    previous stage's controls) and the DISTILLATION family: same sizes,
    Jacobian and Hessian patterns (as sets) and symbolic analysis."""
    H = 7
    pg = N.Problem(N.stage_model_structure(compiled["distillation"], H, 0.1))
    ph = N.Problem(N.distillation_structure(6, H, 0.1, 2.3, F=1.0, rho=0.05))
    assert (pg.n, pg.m_c, pg.m_d, pg.nx, pg.nu, pg.nnz_k) == (ph.n, ph.m_c, ph.m_d, ph.nx, ph.nu, ph.nnz_k)
    pg.analyze()
    ph.analyze()
    a, b = pg.patterns(), ph.patterns()
    for rk, ck in (("j_rows", "j_cols"), ("w_rows", "w_cols")):
        assert set(zip(a[rk].tolist(), a[ck].tolist())) == set(zip(b[rk].tolist(), b[ck].tolist())), rk
    assert pg.symbolic_sizes() == ph.symbolic_sizes()
    assert pg.n_setpoint == 2 and pg.n_traj == H


def _create_rc(s):
    h = C.c_void_p()
    rc = capi.lib().nmpc_create_problem(C.byref(s), C.byref(h))
    if rc == 0:
        capi.lib().nmpc_destroy(h)
    return rc


def test_c_abi_rejects_malformed_descriptors(compiled):
    g = compiled["toy"]
    assert _create_rc(N.stage_model_structure(g, 14, 0.5)) == 0
    bad = []
    s = N.stage_model_structure(g, 14, 0.5)
    s.stage_model.contents.tag = 0
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s._keep[0]["row_cols"][:] = [1, 0]            # not ascending
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s._keep[0]["row_cols"][:] = [1, 1]            # repeated, and the state's own column is missing
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s._keep[0]["lb"][1] = 5.0                     # lb > ub of u
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s._keep[0]["w_rows"][:] = [0, 0]              # upper entry (0, 1) and repeated (0, 0)
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s._keep[0]["prev_coef"][:] = [0.0]            # zero coefficient
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s.control_horizon = 3
    bad.append(s)
    s = N.stage_model_structure(g, 0, 0.5)        # empty horizon
    bad.append(s)
    s = N.stage_model_structure(g, 14, -1.0)
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s.stage_model.contents.code_object_size = 0
    bad.append(s)
    s = N.stage_model_structure(g, 14, 0.5)
    s.stage_model = None
    bad.append(s)
    for i, s in enumerate(bad):
        assert _create_rc(s) == capi.NMPC_ERR_INVALID_ARG, i
    # an algebraic row may not use previous states
    gr = compiled["reflux"]
    s = N.stage_model_structure(gr, 4, 2.0)
    pp = s._keep[0]["prev_ptr"]
    assert pp[8] == pp[-1]                       # rows 8.. (algebraic) hold none
    s._keep[0]["prev_ptr"][9:] += 1              # give row 8 one previous column (reusing an index)
    assert _create_rc(s) == capi.NMPC_ERR_INVALID_ARG
