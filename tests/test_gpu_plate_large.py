"""GPU parity of the heated plate at the sizes where the multi-workgroup
large-front path runs several 512-column outer panels, and the differentiated
workload at full size.

* 32 x 32 grid, horizon 16 (n = 16,640), under the family (lattice)
  dissection: the top time separator is a 1,024-column supernode with 1,536
  rows, below it fronts of 512 and 448 columns.  Cold solve, warm re-solve and sensitivities are compared with the
  oracle entry by entry.
* 64 x 64 grid, horizon 100 (n = 411,200), the differentiated workload: no
  oracle solve is feasible (its dense factor alone would take 1.35 TB), so the
  GPU solution is certified instead.  The oracle's own evaluator recomputes the
  KKT error of the original problem (eqs. 7-9) from the downloaded solution,
  the setpoint gradient is pinned by the envelope theorem (the target enters
  only the objective), and sampled directions of d u1 / d x0 are pinned by
  central differences (h = 1e-6) of re-solves of the same barrier problem,
  converged tightly with the fixed-barrier option."""
import sys

import numpy as np
import pytest

from oracle.adjoint import sensitivities
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate import PlateOCP
from paper_2606_04725_amd import nmpc as N
from workloads import plate_workload
from plate_parity import PARITY_TOL, certify, close, compare_tight, note, tighten_gpu, tighten_ref

pytestmark = pytest.mark.gpu

# Iteration counts of the 32 x 32 x 16 cold solve are not fixed by FP64
# arithmetic: at mu = 1.84e-6 the filter line search spends a long stretch of
# short steps whose accept/reject decisions are near-ties, and the oracle
# itself takes 46 iterations from the cold start and 32, 33, 33, 33 from
# starts perturbed by 1e-15 relative (four seeds).  The counts are only held
# to that spread; the points are compared after tightening.
ITERS_SLACK_32 = 16

_note = note
_close = close


def _problem(w, m):
    # 32 x 32 x 16 under the plate family's own (lattice) dissection, whose
    # fronts the module docstring lists; the 64 x 64 x 100 workload under the
    # default ordering the bench uses
    o = N.capi.NMPC_ORDER_FAMILY_DISSECTION if w.G == 32 else N.capi.NMPC_ORDER_NESTED_DISSECTION
    p = N.Problem(N.plate_structure(w.G, w.H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi, ordering=o))
    p.analyze()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    return p


@pytest.fixture(scope="module")
def plate32():
    """The oracle's cold solve, its tightening on the final barrier problem,
    sensitivities there, plant step, warm re-solve and its tightening, for the
    32 x 32 x 16 plate (a few minutes of host time, computed once)."""
    w = plate_workload("large", 0, G=32, H=16)
    m = PlateOCP.from_workload(w)
    ipm = LiftedIPM(m, IPMOptions(tol=PARITY_TOL))
    _note("plate 32x32x16: oracle cold solve")
    log = lambda it, mu, E0: _note(f"oracle iteration {it}: mu {mu:.2e}, E0 {E0:.2e}")
    cold = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold, progress=log)
    assert cold.status == 0
    _note(f"oracle cold: {cold.iters} iterations; tightening")
    cold_t = tighten_ref(ipm, cold)
    _note("oracle sensitivities")
    sens = sensitivities(ipm, cold_t.state)
    x1 = m.step(m.x0, m.u1(cold_t.state.y))
    m.set_parameters(x0=x1)
    _note("oracle warm re-solve")
    warm = ipm.solve(cold_t.state, ipm.o.mu0_warm, progress=log)
    assert warm.status == 0
    _note(f"oracle warm: {warm.iters} iterations; tightening")
    warm_t = tighten_ref(ipm, warm)
    m.set_parameters(x0=w.T0)
    return dict(w=w, m=m, ipm=ipm, cold=cold, cold_t=cold_t, sens=sens, x1=x1, warm=warm, warm_t=warm_t)


@pytest.mark.timeout(900)
def test_plate32_fronts_exceed_one_outer_panel(plate32):
    w, m = plate32["w"], plate32["m"]
    p = _problem(w, m)
    sym = p.export_symbolic()
    width = np.diff(sym["snode_ptr"])
    assert width.max() == 1024 and np.sum(width > 512) >= 1


@pytest.mark.timeout(900)
def test_plate32_cold_and_warm_match_oracle(plate32):
    w, m, ipm = plate32["w"], plate32["m"], plate32["ipm"]
    p = _problem(w, m)
    gopts = N.default_options(tol=PARITY_TOL)
    _note("plate 32x32x16: gpu cold solve")
    r = p.solve(warm=False, options=gopts)
    assert r.status == 0
    m.set_parameters(x0=w.T0)
    certify(m, ipm, p.solution(), r, plate32["cold"], ITERS_SLACK_32)
    tighten_gpu(p, r.mu)
    compare_tight(m, p.solution(), plate32["cold_t"])
    _note("gpu warm re-solve")
    p.set_parameters(plate32["x1"])
    r2 = p.solve(warm=True, options=gopts)
    assert r2.status == 0
    m.set_parameters(x0=plate32["x1"])
    try:
        certify(m, ipm, p.solution(), r2, plate32["warm"], ITERS_SLACK_32)
        tighten_gpu(p, r2.mu)
        compare_tight(m, p.solution(), plate32["warm_t"])
    finally:
        m.set_parameters(x0=w.T0)


@pytest.mark.timeout(900)
def test_plate32_sensitivities_match_oracle(plate32):
    w, m, sens, st = plate32["w"], plate32["m"], plate32["sens"], plate32["cold_t"].state
    p = _problem(w, m)
    _note("plate 32x32x16: gpu cold solve, tightened, sensitivities at its own solution")
    r = p.solve(warm=False, options=N.default_options(tol=PARITY_TOL))
    assert r.status == 0
    tighten_gpu(p, r.mu)
    rng = np.random.default_rng(11)
    su, so = rng.normal(size=16), float(rng.normal())
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    assert _close(J, sens["x0"]["du1"], 1e-5)
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "setpoint"):
        assert _close(g[key], su @ sens[key]["du1"] + so * sens[key]["df"], 1e-5), key
    _note("sensitivities at the oracle's solution")
    p.set_iterate(st.y, st.s, st.omega, st.beta, st.zL, st.zU)
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    assert _close(J, sens["x0"]["du1"], 1e-6)
    rc, g = p.adjoint(su, so)
    assert rc == 0
    for key in ("x0", "setpoint"):
        assert _close(g[key], su @ sens[key]["du1"] + so * sens[key]["df"], 1e-6), key


@pytest.mark.timeout(900)
def test_plate_64x64x100_certified():
    w = plate_workload("adjoint", 0)
    m = PlateOCP.from_workload(w)
    _note("plate 64x64x100: analyze")
    p = _problem(w, m)
    _note("cold solve")
    r = p.solve(warm=False)
    assert r.status == 0, r.status
    sol = p.solution()
    _note(f"cold: {r.iters} iterations; oracle KKT evaluation")
    e = kkt_error(m, sol["y"], sol["lam"], np.zeros(0), sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
    x1 = m.step(m.x0, sol["u1"])
    m.set_parameters(x0=x1)
    p.set_parameters(x1)
    _note("warm re-solve")
    r2 = p.solve(warm=True)
    assert r2.status == 0, r2.status
    sol = p.solution()
    e = kkt_error(m, sol["y"], sol["lam"], np.zeros(0), sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
    # the barrier problem at the final mu, converged tightly (Newton at fixed mu)
    fo = N.default_options(fixed_mu=1, tol=1e-13, mu0_warm=r2.mu, max_iter=25)
    _note("fixed-barrier tightening")
    rt = p.solve(warm=True, options=fo)
    _note(f"tightened: status {rt.status}, {rt.iters} iterations")
    assert rt.status == 0
    base = p.get_iterate()
    rc, J = p.jacobian_u1_x0()
    assert rc == 0
    rc, g = p.adjoint(np.zeros(16), 1.0)
    assert rc == 0
    # envelope theorem: the target enters only f, so df*/dT*_p = -2 sum_k (T_kp - T*_p)
    # up to barrier and lifting terms of order mu and gamma
    T = base["y"].reshape(m.H, m.ns)[:, :m.nx]
    partial = -2.0 * np.sum(T - m.target[None, :], axis=0)
    assert np.max(np.abs(g["setpoint"] - partial)) <= 1e-5 * max(1.0, np.max(np.abs(partial)))
    # central differences of re-solves from the tightened point, on sampled directions of x0
    rng = np.random.default_rng(7)
    dirs = []
    for j in rng.choice(m.nx, 2, replace=False):
        v = np.zeros(m.nx)
        v[j] = 1.0
        dirs.append(v)
    v = rng.normal(size=m.nx)
    dirs.append(v / np.max(np.abs(v)))
    h = 1e-6
    for k, v in enumerate(dirs):
        us = []
        for sgn in (+1.0, -1.0):
            p.set_parameters(x1 + sgn * h * v)
            p.set_iterate(base["y"], base["s"], base["omega"], base["beta"], base["zL"], base["zU"])
            rs = p.solve(warm=True, options=fo)
            assert rs.status == 0, (k, sgn, rs.status)
            us.append(p.first_stage()[0])
        fd = (us[0] - us[1]) / (2.0 * h)
        jv = J @ v
        _note(f"direction {k}: |J v - fd| {np.max(np.abs(jv - fd)):.3e}, |fd| {np.max(np.abs(fd)):.3e}")
        assert np.max(np.abs(jv - fd)) <= 1e-5 * max(1e-3, np.max(np.abs(fd))) + 1e-7, k
