"""GPU sensitivities (implicit function theorem on the lifted barrier KKT
conditions, condensed as eqs. 14 and 17) against the oracle at the same iterate."""
import sys

import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.distillation import DistillationOCP
from oracle.ipm import LiftedIPM
from paper_2606_04725_amd import nmpc as N
from workloads import distillation_workload

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _setup(name, seed, **over):
    w = distillation_workload(name, seed, **over)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    st = res.state
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    return w, m, ipm, st, p


# Both sides solve the uncondensed sensitivity system (the oracle by sparse LU,
# the library by its Cholesky of the condensed matrix refined against the
# uncondensed residual), so they agree well below the 1e-5 sensitivity bar.
TOL = 1e-6


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) / max(1.0, float(np.max(np.abs(b))))


@pytest.mark.parametrize("name,seed", [("small", 0), ("small", 3), ("medium", 0)])
def test_adjoint_matches_oracle(name, seed):
    _note(f"adjoint {name} seed={seed}")
    w, m, ipm, st, p = _setup(name, seed)
    sens = sensitivities(ipm, st)
    rng = np.random.default_rng(seed)
    su, so = rng.normal(size=2), float(rng.normal())
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key, ref_key in (("x0", "x0"), ("setpoint", "setpoint"), ("traj", "zF"), ("u_prev", "u_prev")):
        ref = su @ sens[ref_key]["du1"] + so * sens[ref_key]["df"]
        assert _rel(g[key], ref) <= TOL, (key, _rel(g[key], ref))
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    assert _rel(J, sens["x0"]["du1"]) <= TOL


def test_adjoint_after_solve_and_repeat_calls():
    _note("adjoint after a GPU solve, repeated calls reuse the factor")
    w = distillation_workload("small", 1)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    r = p.solve()
    assert r.status == 0
    _, g1 = p.adjoint(np.array([1.0, 0.0]), 0.0)
    _, g2 = p.adjoint(np.array([1.0, 0.0]), 0.0)
    for k in g1:
        assert np.array_equal(g1[k], g2[k])
    _, J = p.jacobian_u1_x0()
    assert np.allclose(J[0], g1["x0"], rtol=1e-12, atol=1e-15)


def _plate_problem(G, H):
    from workloads import plate_workload
    w = plate_workload("large", 0, G=G, H=H)
    p = N.Problem(N.plate_structure(G, H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
    p.analyze()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=np.full(16, 0.5))
    return p


@pytest.mark.parametrize("family", ["distillation", "plate"])
def test_jacobian_rows_are_the_seeded_adjoints(family):
    """The Jacobian solves its nu seeds together (one batch of launches over
    instances that share the factor); row k must be exactly what the
    single-seed adjoint returns for e_k.  The 16 x 10 plate has supernodes on
    the multi-workgroup solve path, so its launches carry tasks of every seed."""
    _note(f"jacobian rows against seeded adjoints, {family}")
    if family == "distillation":
        w = distillation_workload("small", 1)
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    else:
        p = _plate_problem(16, 10)
    r = p.solve()
    assert r.status == 0
    for rep in range(2):   # the seed batch is built on the first call and reused
        rc, J = p.jacobian_u1_x0()
        assert rc == 0
        for k in range(p.nu):
            e = np.zeros(p.nu)
            e[k] = 1.0
            _, g = p.adjoint(e, 0.0)
            assert np.array_equal(J[k], g["x0"]), (rep, k, float(np.max(np.abs(J[k] - g["x0"]))))


def test_autograd_function():
    _note("torch autograd")
    import torch
    from paper_2606_04725_amd.autograd import NMPCSolve
    w, m, ipm, st, p = _setup("small", 2)
    x0 = torch.tensor(w.x0, dtype=torch.float64, requires_grad=True)
    sp = torch.tensor([w.xD_sp, w.xB_sp], dtype=torch.float64, requires_grad=True)
    tr = torch.tensor(w.zF(0), dtype=torch.float64)
    up = torch.tensor(w.u_prev0, dtype=torch.float64)
    u1, f = NMPCSolve.apply(p, x0, sp, tr, up, True)
    loss = 2.0 * u1[0] - u1[1] + 0.5 * f
    loss.backward()
    # reference: the oracle's sensitivities at its own solution of the same
    # parameters (the forward re-solved warm from that point on the GPU)
    sens = sensitivities(ipm, st)
    ref_x0 = np.array([2.0, -1.0]) @ sens["x0"]["du1"] + 0.5 * sens["x0"]["df"]
    assert _rel(x0.grad.numpy(), ref_x0) <= 1e-5
    ref_sp = np.array([2.0, -1.0]) @ sens["setpoint"]["du1"] + 0.5 * sens["setpoint"]["df"]
    assert _rel(sp.grad.numpy(), ref_sp) <= 1e-5


def test_sensitivities_refuse_a_changed_problem():
    """The handle holds one solution: after new parameters (without a solve) the
    sensitivity entry points refuse, and an autograd backward whose forward's
    solution has been replaced raises instead of differentiating another
    solution."""
    _note("stale sensitivities are refused")
    import torch
    from paper_2606_04725_amd import capi
    from paper_2606_04725_amd.autograd import NMPCSolve
    w = distillation_workload("small", 1)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    assert p.solve().status == 0
    sid, cur = p.solution_id()
    assert cur and sid >= 1
    p.set_parameters(w.x0 + 1e-3, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    assert p.solution_id() == (sid, False)
    for call in (lambda: p.adjoint(np.ones(2), 0.0), p.jacobian_u1_x0):
        with pytest.raises(N.NMPCError) as e:
            call()
        assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    assert p.solve(warm=True).status == 0
    assert p.solution_id() == (sid + 1, True)
    assert p.adjoint(np.ones(2), 0.0)[0] == 0
    # two forwards on one problem, then the first one's backward
    t = lambda v: torch.tensor(v, dtype=torch.float64)  # noqa: E731
    x0a = t(w.x0).requires_grad_(True)
    u1a, _ = NMPCSolve.apply(p, x0a, t([w.xD_sp, w.xB_sp]), t(w.zF(0)), t(w.u_prev0), True)
    x0b = t(w.x0 + 1e-3).requires_grad_(True)
    u1b, _ = NMPCSolve.apply(p, x0b, t([w.xD_sp, w.xB_sp]), t(w.zF(0)), t(w.u_prev0), True)
    with pytest.raises(RuntimeError, match="solved again"):
        u1a.sum().backward()
    u1b.sum().backward()
    assert torch.all(torch.isfinite(x0b.grad))
