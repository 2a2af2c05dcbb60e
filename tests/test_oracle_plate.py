"""Pins for the oracle's heated-plate model and its interior-point solutions:
the ghost-node layout, the discrete maximum principle, the symmetry of the
problem under swapping the two coordinates, and the constant-conductivity case
against the finite-horizon Riccati closed form."""
import numpy as np
import pytest

from oracle.ipm import LiftedIPM
from oracle.kkt import kkt_error
from oracle.plate import PlateOCP, ghost_segments
from oracle.riccati import riccati_gains
from workloads import plate_workload


def _transpose_field(v, G):
    return np.asarray(v).reshape(G, G).T.reshape(-1)


def _transpose_controls(u):
    """Segments under the swap of the two coordinates: bottom <-> left, right <-> top."""
    u = np.asarray(u)
    return np.concatenate([u[12:16], u[8:12], u[4:8], u[0:4]])


def _transpose_y(m, y):
    Y = y.reshape(m.H, m.ns)
    out = np.empty_like(Y)
    for k in range(m.H):
        out[k, :m.nx] = _transpose_field(Y[k, :m.nx], m.G)
        out[k, m.nx:] = _transpose_controls(Y[k, m.nx:])
    return out.reshape(-1)


def test_ghost_segment_layout():
    g = ghost_segments(8)
    assert g[0] == [0, 12]      # (a, b) = (0, 0): bottom segment 0, left segment 0
    assert g[7] == [3, 4]       # (7, 0): bottom segment 3, right segment 0
    assert g[56] == [8, 15]     # (0, 7): top segment 0, left segment 3
    assert g[63] == [7, 11]     # (7, 7): right segment 3, top segment 3
    assert g[9] == []           # interior node (1, 1)
    counts = np.bincount([s for v in g for s in v], minlength=16)
    assert np.all(counts == 2)  # every segment drives G / 4 ghost nodes


def _laplacian_and_heaters(G):
    """Constant-conductivity semi-discretisation written out from scratch:
    dT/dt = (L T + B u) / h^2 with Dirichlet ghost values from the heaters."""
    n = G * G
    L = np.zeros((n, n))
    B = np.zeros((n, 16))
    q = G // 4
    for b in range(G):
        for a in range(G):
            p = b * G + a
            for (da, db) in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                aa, bb = a + da, b + db
                L[p, p] -= 1.0
                if 0 <= aa < G and 0 <= bb < G:
                    L[p, bb * G + aa] += 1.0
                elif bb < 0:
                    B[p, a // q] += 1.0
                elif aa >= G:
                    B[p, 4 + b // q] += 1.0
                elif bb >= G:
                    B[p, 8 + a // q] += 1.0
                else:
                    B[p, 12 + b // q] += 1.0
    return L, B


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_discrete_maximum_principle(sigma):
    G = 8
    m = PlateOCP(G, 1, 0.01, sigma=sigma)
    rng = np.random.default_rng(3)
    for _ in range(3):
        x = rng.uniform(0.0, 1.0, m.nx)
        u = rng.uniform(0.0, 1.0, 16)
        T = m.step(x, u)
        lo, hi = min(x.min(), u.min()), max(x.max(), u.max())
        assert T.min() >= lo - 1e-12 and T.max() <= hi + 1e-12


def test_constant_conductivity_step_is_linear_solve():
    G, dt = 8, 0.01
    m = PlateOCP(G, 1, dt, sigma=0.0)
    L, B = _laplacian_and_heaters(G)
    h2 = m.h ** 2
    rng = np.random.default_rng(4)
    x, u = rng.uniform(size=m.nx), rng.uniform(size=16)
    T = m.step(x, u)
    ref = np.linalg.solve(np.eye(m.nx) - dt * L / h2, x + dt * B @ u / h2)
    assert np.max(np.abs(T - ref)) <= 1e-12


def test_model_commutes_with_coordinate_swap():
    G, H = 8, 3
    m = PlateOCP(G, H, 0.01)
    rng = np.random.default_rng(5)
    y = rng.uniform(0.0, 1.0, m.n)
    x0, tgt = rng.uniform(size=m.nx), rng.uniform(size=m.nx)
    m.set_parameters(x0=x0, target=tgt)
    c, f = m.cons_c(y), m.f(y)
    m.set_parameters(x0=_transpose_field(x0, G), target=_transpose_field(tgt, G))
    ct = m.cons_c(_transpose_y(m, y))
    assert np.allclose(ct.reshape(H, -1), np.array([_transpose_field(v, G) for v in c.reshape(H, -1)]),
                       rtol=0, atol=1e-12)
    assert abs(m.f(_transpose_y(m, y)) - f) <= 1e-12


def test_symmetric_problem_has_symmetric_solution():
    w = plate_workload("large", 0, G=8, H=4)
    m = PlateOCP.from_workload(w)
    tgt = 0.5 * (w.target + _transpose_field(w.target, 8))
    m.set_parameters(target=tgt)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    y = res.state.y
    assert np.max(np.abs(_transpose_y(m, y) - y)) <= 1e-7


def test_constant_conductivity_matches_riccati():
    """sigma = 0 and wide bounds: the plate is an LQ problem with
    A = (I - dt L/h^2)^{-1}, B = A dt Bh/h^2, Q = I, R = 0, so the first
    control is -K_1 x0 + kff_1 (up to the lifting and the barrier)."""
    G, H, dt = 8, 5, 0.01
    m = PlateOCP(G, H, dt, sigma=0.0, t_hi=1e3, c_lo=-1e3, c_hi=1e3)
    rng = np.random.default_rng(6)
    x0, tgt = rng.uniform(0.0, 0.5, m.nx), rng.uniform(0.2, 0.8, m.nx)
    m.set_parameters(x0=x0, target=tgt)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    L, Bh = _laplacian_and_heaters(G)
    h2 = m.h ** 2
    A = np.linalg.inv(np.eye(m.nx) - dt * L / h2)
    B = A @ (dt * Bh / h2)
    K, kff = riccati_gains(A, B, np.eye(m.nx), np.zeros((16, 16)), H, tgt)
    u1 = -K[1] @ x0 + kff[1]
    assert np.max(np.abs(m.u1(res.state.y) - u1)) <= 1e-5 * max(1.0, np.max(np.abs(u1)))


def test_plate_solution_is_kkt_point():
    w = plate_workload("large", 1, G=8, H=5)
    m = PlateOCP.from_workload(w)
    ipm = LiftedIPM(m)
    res = ipm.solve(ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold), ipm.o.mu0_cold)
    assert res.status == 0
    st = res.state
    lam = st.omega[:m.m_c] - st.omega[m.m_c:2 * m.m_c]
    e = kkt_error(m, st.y, lam, np.zeros(0), st.zL, st.zU)
    assert e["max"] <= 1e-8, e
