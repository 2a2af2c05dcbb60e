"""HyKKT variant on the GPU (nmpc_options.kkt = NMPC_KKT_HYKKT) against the
oracle's HyKKT method (oracle/hykkt.py) and the reference route
(oracle/ref_ipm.py), through the C ABI.

Both sides solve cold with an E_0 tolerance only mu_min can meet, their
returned points are certified (KKT error of the original problem, equal
barrier value, iteration counts within two), then each side tightens its own
point on that barrier problem (fixed mu, E_mu <= 1e-12) and the tightened
points are compared entry by entry at 1e-6 (the reason is the one given in
tests/plate_parity.py: near active bounds the stopping ball is wider than
1e-6)."""
import numpy as np
import pytest

from oracle.distillation import DistillationOCP
from oracle.hykkt import HyKKTIPM
from oracle.ipm import IPMOptions
from oracle.kkt import kkt_error
from oracle.plate import PlateOCP
from oracle.ref_ipm import ReferenceIPM
from paper_2606_04725_amd import capi
from paper_2606_04725_amd import nmpc as N
from plate_parity import PARITY_TOL, TIGHT_TOL, note, rel_dev
from workloads import distillation_workload, plate_workload

pytestmark = pytest.mark.gpu


def _hk(**kw):
    return N.default_options(kkt=capi.NMPC_KKT_HYKKT, **kw)


def _case(kind):
    if kind[0] == "column":
        w = distillation_workload(kind[1], kind[2])
        m = DistillationOCP.from_workload(w)
        m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
        p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
        p.analyze()
        p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    else:
        w = plate_workload("large", kind[3], G=kind[1], H=kind[2])
        m = PlateOCP.from_workload(w)
        p = N.Problem(N.plate_structure(w.G, w.H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
        p.analyze()
        p.set_parameters(w.T0, setpoint=w.target, u_prev=m.u_prev)
    return m, p


def _compare(m, ipm, sol, st):
    lam, nu = ipm.multipliers(st)
    for key, got, want in (("y", sol["y"], st.y), ("lam", sol["lam"], lam), ("nu", sol["omega_d"], nu),
                           ("zL", sol["zL"], st.zL), ("zU", sol["zU"], st.zU)):
        if len(want) == 0:
            continue
        d = rel_dev(got, want)
        note(f"tightened {key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


CASES = [("column", "small", 0), ("column", "small", 3), ("column", "medium", 0), ("plate", 8, 5, 1),
         ("plate", 16, 10, 0)]


@pytest.mark.parametrize("kind", CASES, ids=lambda k: "-".join(map(str, k)))
def test_hykkt_cold_solve_matches_oracle(kind):
    note(f"HyKKT cold solve {kind}")
    m, p = _case(kind)
    ipm = HyKKTIPM(m, IPMOptions(tol=PARITY_TOL))
    ref = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert ref.status == 0
    r = p.solve(warm=False, options=_hk(tol=PARITY_TOL))
    note(f"iterations gpu {r.iters} oracle {ref.iters}; CG gpu {r.cg_iters} oracle {ipm.cg_total}; "
         f"mu gpu {r.mu:.2e} oracle {ref.mu:.2e}")
    assert r.status == 0
    assert r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min
    assert abs(r.iters - ref.iters) <= 2
    assert 0 < r.cg_iters <= 20 * r.iters
    sol = p.solution()
    e = kkt_error(m, sol["y"], sol["lam"], sol["omega_d"], sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
    rt = p.solve(warm=True, options=_hk(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=r.mu, max_iter=30))
    assert rt.status == 0
    ref_t = ipm.solve(ref.state, ref.mu, fixed_mu=True, tol=TIGHT_TOL)
    assert ref_t.status == 0
    _compare(m, ipm, p.solution(), ref_t.state)


@pytest.mark.parametrize("seed", [0, 4])
def test_hykkt_reaches_the_reference_point(seed):
    """The KKT point of the problem as posed: the reference route (dense
    LDL^T, no lifting) at tol 1e-10 against the GPU's HyKKT solve at tol 1e-10,
    mu_min 1e-11 (no relaxation parameter involved), cold and warm from a
    Lifted-KKT solution at the default options."""
    note(f"HyKKT vs reference route, small column seed {seed}")
    m, p = _case(("column", "small", seed))
    ref = ReferenceIPM(m).solve(m.initial_guess())
    assert ref.status == 0
    sy, sl = max(1.0, np.max(np.abs(ref.y))), max(1.0, np.max(np.abs(ref.lam)))
    tight = dict(tol=1e-10, mu_min=1e-11, mu0_warm=1e-11)
    for warm in (False, True):
        if warm:
            assert p.solve(warm=False).status == 0      # Lifted-KKT, default options
        r = p.solve(warm=warm, options=_hk(**tight))
        assert r.status == 0, r.status
        s = p.solution()
        note(f"warm {warm}: {r.iters} iterations, |y - ref| {np.max(np.abs(s['y'] - ref.y)):.2e}")
        assert np.max(np.abs(s["y"] - ref.y)) / sy <= 1e-6
        assert np.max(np.abs(s["lam"] - ref.lam)) / sl <= 1e-6
        assert np.max(np.abs(s["omega_d"] - ref.nu)) / max(1.0, np.max(np.abs(ref.nu))) <= 1e-6


def test_hykkt_api_rules():
    """HyKKT solves one problem at a time; its solutions have no sensitivities
    and no warm Lifted-KKT continuation (a cold one is fine)."""
    note("HyKKT API rules")
    m, p = _case(("column", "small", 2))
    assert p.solve(warm=False, options=_hk()).status == 0
    with pytest.raises(N.NMPCError) as e:
        p.adjoint(np.ones(2), 0.0)
    assert e.value.code == -2   # NMPC_ERR_BAD_ORDER
    with pytest.raises(N.NMPCError):
        p.solve(warm=True)
    assert p.solve(warm=False).status == 0
    rc, _ = p.adjoint(np.ones(2), 0.0)
    assert rc == 0
    b = N.Batch([p])
    with pytest.raises(N.NMPCError):
        b.solve(warm=False, options=_hk())
    b.close()
