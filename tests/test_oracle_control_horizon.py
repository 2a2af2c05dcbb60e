"""Control horizon of the distillation model (Section 3.1, eqs. 4-5), oracle
side: the hold rows are the differences of consecutive controls past the
control horizon (checked entry by entry against index arithmetic on y and by
complex-step derivatives), and both interior-point routes return points that
hold the controls, satisfy the KKT conditions of the held problem and cost at
least the free problem's optimum."""
import numpy as np
import pytest

from oracle.distillation import DistillationOCP
from oracle.hykkt import HyKKTIPM
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from workloads import distillation_workload


def _model(Hc, kind="small", seed=0):
    w = distillation_workload(kind, seed, Hc=Hc)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    return m


def test_hold_rows_by_index():
    m = _model(5)
    assert m.m_c == m.H * m.nx + 2 * (m.H - 5)
    y = np.random.default_rng(0).uniform(0.5, 2.0, m.n)
    c = m.cons_c(y)
    tail = c[m.H * m.nx:].reshape(m.H - 5, 2)
    for k in range(5, m.H):
        assert tail[k - 5, 0] == y[k * m.ns + m.nx] - y[(k - 1) * m.ns + m.nx]
        assert tail[k - 5, 1] == y[k * m.ns + m.nx + 1] - y[(k - 1) * m.ns + m.nx + 1]
    # the dynamics rows are those of the free model
    assert np.array_equal(c[:m.H * m.nx], _model(0).cons_c(y))


def test_hold_jacobian_complex_step():
    m = _model(7)
    rng = np.random.default_rng(1)
    y = rng.uniform(0.2, 0.8, m.n)
    y[m.nx::m.ns] = rng.uniform(1.0, 3.0, m.H)
    y[m.nx + 1::m.ns] = rng.uniform(1.0, 3.0, m.H)
    J = m.jac_c(y).toarray()
    h = 1e-30
    for j in rng.choice(m.n, 40, replace=False):
        e = np.zeros(m.n, dtype=complex)
        e[j] = 1j * h
        assert np.allclose(np.imag(m.cons_c(y + e)) / h, J[:, j], rtol=0, atol=1e-13)


@pytest.mark.parametrize("route", ["lifted", "hykkt"])
def test_held_solution(route):
    Hc = 5
    m, free = _model(Hc), _model(0)
    make = (lambda mm: LiftedIPM(mm)) if route == "lifted" else (lambda mm: HyKKTIPM(mm))
    ipm, ipf = make(m), make(free)
    r = ipm.solve(ipm.cold_start(m.initial_guess(), 0.1), 0.1)
    rf = ipf.solve(ipf.cold_start(free.initial_guess(), 0.1), 0.1)
    assert r.status == 0 and rf.status == 0
    y = r.state.y
    U = y.reshape(m.H, m.ns)[:, m.nx:]
    assert np.max(np.abs(U[Hc:] - U[Hc - 1])) <= 1e-7        # held at stage Hc's control
    assert np.max(np.abs(np.diff(rf.state.y.reshape(m.H, m.ns)[:, m.nx:], axis=0))) > 1e-3   # the free one moves
    lam, nu = ipm.multipliers(r.state)
    assert kkt_error(m, y, lam, nu, r.state.zL, r.state.zU)["max"] <= 1e-8
    assert m.f(y) >= free.f(rf.state.y) - 1e-8


@pytest.mark.parametrize("Hc", [0, 6])
def test_shift_state_by_index(Hc):
    """The shifted warm start moves every stage-indexed entry one stage
    earlier: checked against explicit index arithmetic on random data."""
    from oracle.ipm import IPMState
    from oracle.nmpc import shift_state
    m = _model(Hc)
    rng = np.random.default_rng(4)
    ml = 2 * m.m_c + m.m_d
    st = IPMState(*(rng.normal(size=k) for k in (m.n, ml, ml, ml, m.n, m.n)))
    sh = shift_state(m, st)
    H, nx, ns, mc = m.H, m.nx, m.ns, m.m_c
    for k in range(H):
        src = k + 1 if k < H - 1 else k
        assert np.array_equal(sh.y[k * ns:(k + 1) * ns], st.y[src * ns:(src + 1) * ns])
        assert np.array_equal(sh.zU[k * ns:(k + 1) * ns], st.zU[src * ns:(src + 1) * ns])
        for off in (0, mc):
            assert np.array_equal(sh.omega[off + k * nx:off + (k + 1) * nx],
                                  st.omega[off + src * nx:off + (src + 1) * nx])
        assert np.array_equal(sh.s[2 * mc + 2 * k:2 * mc + 2 * k + 2], st.s[2 * mc + 2 * src:2 * mc + 2 * src + 2])
    hc = m.Hc
    for k in range(hc, H):                     # hold rows of stage k (two each)
        src = k + 1 if k < H - 1 else k
        for off in (0, mc):
            a = off + H * nx + 2 * (k - hc)
            b = off + H * nx + 2 * (src - hc)
            assert np.array_equal(sh.beta[a:a + 2], st.beta[b:b + 2])


def test_shift_state_by_index_with_algebraic_rows():
    """The case-study column (Section 4.1) has 2 N + 3 equality rows per stage
    (tray balances, equilibrium rows, flow rows): all of a stage's rows move
    together, checked against explicit index arithmetic on random data."""
    from oracle.ipm import IPMState
    from oracle.nmpc import shift_state
    from oracle.reflux import RefluxColumnOCP
    m = RefluxColumnOCP(5, N=6, Nf=3)
    rng = np.random.default_rng(6)
    ml = 2 * m.m_c + m.m_d
    st = IPMState(*(rng.normal(size=k) for k in (m.n, ml, ml, ml, m.n, m.n)))
    sh = shift_state(m, st)
    H, rps, ns, mc = m.H, m.rps, m.ns, m.m_c
    assert rps == 2 * 6 + 3 and mc == H * rps
    for k in range(H):
        src = k + 1 if k < H - 1 else k
        assert np.array_equal(sh.y[k * ns:(k + 1) * ns], st.y[src * ns:(src + 1) * ns])
        for v, w in ((sh.s, st.s), (sh.omega, st.omega), (sh.beta, st.beta)):
            for off in (0, mc):
                assert np.array_equal(v[off + k * rps:off + (k + 1) * rps], w[off + src * rps:off + (src + 1) * rps])
