"""Pins for the oracle's model functions: complex-step derivatives and invariants."""
import numpy as np
import pytest

from oracle.distillation import DistillationOCP
from oracle.lq import LQOCP, random_lq
from oracle.plate import PlateOCP
from oracle.toy import ToyOCP

H_CS = 1e-30


def _rand_point(m, rng):
    y = rng.uniform(0.1, 0.9, m.n)
    if isinstance(m, DistillationOCP):
        for k in range(m.H):
            y[m.iR(k)] = rng.uniform(0.6, 4.0)
            y[m.iV(k)] = rng.uniform(0.6, 4.0)
    return y


def _models():
    rng = np.random.default_rng(7)
    d = DistillationOCP(7, 4, 0.1, 2.3)
    d.set_parameters(x0=rng.uniform(0.1, 0.9, d.nx), zF=rng.uniform(0.4, 0.6, d.H),
                     u_prev=[1.5, 2.2], setpoint=[0.93, 0.07])
    A, B, Q, R, x0, xs = random_lq(3, 2, 4, seed=1)
    lq = LQOCP(A, B, Q, R, 4, xs=xs)
    lq.set_parameters(x0=x0)
    toy = ToyOCP()
    toy.set_parameters(y0=0.7, tk=1.0)
    pl = PlateOCP(8, 3, 0.01)
    pl.set_parameters(x0=rng.uniform(0.0, 0.5, pl.nx), target=rng.uniform(0.2, 0.8, pl.nx))
    return [d, lq, toy, pl]


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_complex_step_derivatives(which):
    m = _models()[which]
    rng = np.random.default_rng(11)
    y = _rand_point(m, rng)
    E = np.eye(m.n)
    # gradient and Jacobian: complex step is exact to rounding for analytic functions
    g_cs = np.array([m.f(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)])
    assert np.max(np.abs(m.grad(y) - g_cs)) <= 1e-13 * max(1.0, np.max(np.abs(g_cs)))
    J_cs = np.array([m.cons_c(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)]).T
    J = m.jac_c(y).toarray()
    assert np.max(np.abs(J - J_cs)) <= 1e-13 * max(1.0, np.max(np.abs(J_cs)))
    if m.m_d:
        Jd_cs = np.array([m.cons_d(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)]).T
        assert np.max(np.abs(m.jac_d(y).toarray() - Jd_cs)) <= 1e-14
    # Hessian of the Lagrangian: complex step of the analytic Lagrangian gradient
    lam = rng.normal(size=m.m_c)
    lam_d = rng.normal(size=m.m_d)

    def grad_L(yy):
        out = m.grad(yy) + m.jac_c(yy).T @ lam
        if m.m_d:
            out = out + m.jac_d(yy).T @ lam_d
        return out
    W_cs = np.array([grad_L(y + 1j * H_CS * E[i]).imag / H_CS for i in range(m.n)]).T
    W = m.hess(y, lam, lam_d).toarray()
    assert np.max(np.abs(W - W_cs)) <= 1e-13 * max(1.0, np.max(np.abs(W_cs)))
    assert np.array_equal(W, W.T)


def test_hessian_central_differences():
    """Second pin on W, independent of complex arithmetic: central differences of
    the Lagrangian gradient built from the Jacobian."""
    m = _models()[0]
    rng = np.random.default_rng(3)
    y = _rand_point(m, rng)
    lam = rng.normal(size=m.m_c)
    h = 1e-6
    W = m.hess(y, lam, np.zeros(m.m_d)).toarray()
    Wfd = np.zeros_like(W)
    for i in range(m.n):
        e = np.zeros(m.n)
        e[i] = h
        gp = m.grad(y + e) + m.jac_c(y + e).T @ lam
        gm = m.grad(y - e) + m.jac_c(y - e).T @ lam
        Wfd[:, i] = (gp - gm) / (2 * h)
    assert np.max(np.abs(W - Wfd)) < 1e-7


def test_structural_pattern_covers_values():
    m = _models()[0]
    y = _rand_point(m, np.random.default_rng(5))
    J = m.jac_c(y)
    assert J.nnz == len(m.jc_rows)    # every structural entry is stored
    dense = J.toarray()
    mask = np.zeros_like(dense, dtype=bool)
    mask[m.jc_rows, m.jc_cols] = True
    assert np.all(dense[~mask] == 0.0)


def test_distillation_component_balance():
    """Sum of holdup derivatives equals feed in minus distillate and bottoms out:
    sum_i dx_i/dt = F zF - D x_0 - B x_{N+1}."""
    m = DistillationOCP(9, 6, 0.1, 2.7)
    rng = np.random.default_rng(2)
    X = rng.uniform(0.05, 0.95, (m.H, m.nx))
    R = rng.uniform(0.6, 3.0, m.H)
    V = R + rng.uniform(0.1, 1.0, m.H)
    zF = rng.uniform(0.3, 0.7, m.H)
    rhs = m.rhs(X, R, V, zF)
    D = V - R
    B = R + m.F - V
    assert np.allclose(rhs.sum(axis=1), m.F * zF - D * X[:, 0] - B * X[:, -1], atol=1e-13)


def test_distillation_total_reflux_fixed_point():
    """With F = 0 and R = V (total reflux, no product flows) the uniform profile
    x = y(x) can only hold at x in {0, 1}; the profile with every tray vapor in
    equilibrium with the liquid above is a fixed point of the tray equations."""
    m = DistillationOCP(5, 1, 0.1, 2.0, F=0.0)
    a = m.alpha
    # build x top-down: x_0 = y(x_1) from the condenser, tray i: x_{i-1} = y(x_i)
    x = np.zeros(m.nx)
    x[-1] = 0.2
    for i in range(m.nx - 2, -1, -1):
        x[i] = a * x[i + 1] / (1 + (a - 1) * x[i + 1])
    R = V = np.array([1.7])
    rhs = m.rhs(x[None, :], R, V, np.zeros(1))
    assert np.max(np.abs(rhs)) < 1e-14
