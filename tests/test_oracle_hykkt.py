"""The oracle's HyKKT interior-point method (oracle/hykkt.py), pinned against
routes it shares no linear algebra with:

* the HyKKT solve of the condensed system (Cholesky of K_c + gamma_h J_c^T J_c
  and CG on the Schur complement) equals a sparse LU solve of the 2 x 2 block
  system of eq. (14), at a cold start with random multipliers;
* its solution is the original problem's KKT point: equal to the dense-LDL^T
  reference method (oracle/ref_ipm.py, an independent implementation) and to
  the Riccati closed form of a linear-quadratic problem, and certified by the
  independent KKT evaluator;
* started from a Lifted-KKT solution it removes the lifting's O(gamma + mu)
  offset in a few iterations."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.distillation import DistillationOCP
from oracle.hykkt import HyKKTIPM, HyKKTOptions, hykkt_solve
from oracle.ipm import IPMOptions, LiftedIPM
from oracle.kkt import kkt_error
from oracle.lq import LQOCP, random_lq
from oracle.plate import PlateOCP
from oracle.ref_ipm import ReferenceIPM
from oracle.riccati import riccati_solution
from workloads import distillation_workload, plate_workload


def _column(kind, seed):
    w = distillation_workload(kind, seed)
    m = DistillationOCP.from_workload(w)
    m.set_parameters(x0=w.x0, zF=w.zF(0), u_prev=w.u_prev0)
    return m


def _kkt(m, ipm, st):
    lam, nu = ipm.multipliers(st)
    return kkt_error(m, st.y, lam, nu, st.zL, st.zU)["max"]


@pytest.mark.parametrize("case", ["column", "plate"])
def test_hykkt_solve_equals_block_lu(case):
    m = _column("small", 0) if case == "column" else PlateOCP.from_workload(plate_workload("large", 0, G=8, H=3))
    ipm = HyKKTIPM(m)
    st = ipm.cold_start(m.initial_guess(), 0.1)
    st.omega = np.random.default_rng(3).normal(scale=0.3, size=ipm.ml)
    y = st.y
    step = ipm.newton_step(st, 0.1, m.f(y), m.grad(y), m.cons_c(y), m.cons_d(y), m.jac_c(y), m.jac_d(y))
    assert step["cg_ok"] and step["cg_iters"] <= 20
    Jc = m.jac_c(y)
    A = sp.bmat([[step["K"], Jc.T], [Jc, None]]).tocsc()
    # the right-hand side of eq. (14), rebuilt from the residuals
    r1, r2, Q, _, Jd, *_ = ipm._soc_ctx
    b1 = -r1 - (Jd.T @ (Q * step["r4"][m.m_c:] - r2) if m.m_d else 0.0)
    ref = spla.splu(A).solve(np.concatenate([b1, -m.cons_c(y)]))
    dlam = step["domega"][:m.m_c]
    # K_gamma's condition number grows with gamma_h |J_c|^2 (about 1e8 for the
    # plate), which bounds the solve's accuracy
    assert np.max(np.abs(step["dy"] - ref[:m.n])) <= 1e-8 * max(1.0, np.max(np.abs(ref[:m.n])))
    assert np.max(np.abs(dlam - ref[m.n:])) <= 1e-8 * max(1.0, np.max(np.abs(ref[m.n:])))


def test_hykkt_solve_on_a_random_saddle_system():
    """K positive definite on the null space of H only (indefinite itself):
    the augmented matrix K + gamma H^T H is positive definite and the HyKKT
    solution equals the dense solve."""
    rng = np.random.default_rng(0)
    n, m = 30, 12
    H = rng.normal(size=(m, n))
    Z = np.linalg.svd(H)[2][m:].T                      # null-space basis
    K = Z @ np.diag(rng.uniform(1, 3, n - m)) @ Z.T - H.T @ np.diag(rng.uniform(0.1, 1, m)) @ H
    assert np.min(np.linalg.eigvalsh(K)) < 0
    b1, b2 = rng.normal(size=n), rng.normal(size=m)

    class Dense:
        def solve(self, b):
            return np.linalg.solve(self.K, b)

    chol = Dense()
    chol.K = K + 1e4 * H.T @ H
    np.linalg.cholesky(chol.K)
    dy, dl, it, ok = hykkt_solve(chol, sp.csr_matrix(H), b1, b2, 1e4, 1e-13, 100)
    ref = np.linalg.solve(np.block([[K, H.T], [H, np.zeros((m, m))]]), np.concatenate([b1, b2]))
    assert ok
    assert np.allclose(dy, ref[:n], atol=1e-9) and np.allclose(dl, ref[n:], atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_hykkt_method_reaches_the_reference_point(seed):
    m = _column("small", seed)
    ipm = HyKKTIPM(m, IPMOptions(tol=1e-10, mu_min=1e-12))
    r = ipm.solve(ipm.cold_start(m.initial_guess(), 0.1), 0.1)
    assert r.status == 0
    ref = ReferenceIPM(m).solve(m.initial_guess())
    assert ref.status == 0
    lam, nu = ipm.multipliers(r.state)
    assert np.max(np.abs(r.state.y - ref.y)) <= 1e-7
    assert np.max(np.abs(lam - ref.lam)) <= 1e-7
    assert _kkt(m, ipm, r.state) <= 1e-9


def test_hykkt_method_matches_riccati():
    A, B, Q, R, x0, xs = random_lq(4, 2, 12, seed=3)
    m = LQOCP(A, B, Q, R, 12, xs=xs)
    m.set_parameters(x0=x0)
    ipm = HyKKTIPM(m, IPMOptions(tol=1e-10, mu_min=1e-12))
    r = ipm.solve(ipm.cold_start(m.initial_guess(), 0.1), 0.1)
    assert r.status == 0
    X, U = riccati_solution(A, B, Q, R, 12, x0, xs)
    Y = r.state.y.reshape(12, 6)
    assert np.max(np.abs(Y[:, 4:] - U)) <= 1e-8 * max(1.0, np.max(np.abs(U)))
    assert np.max(np.abs(Y[:, :4] - X)) <= 1e-8 * max(1.0, np.max(np.abs(X)))


@pytest.mark.parametrize("case", ["medium", "plate"])
def test_hykkt_method_default_tolerances(case):
    """40-tray column and 16 x 16 x 10 plate from cold starts: converged with a
    KKT error of the original problem <= 1e-8 and a few CG iterations per
    Newton step."""
    m = _column("medium", 0) if case == "medium" else PlateOCP.from_workload(plate_workload("large", 0, G=16, H=10))
    ipm = HyKKTIPM(m)
    r = ipm.solve(ipm.cold_start(m.initial_guess(), 0.1), 0.1)
    assert r.status == 0 and r.iters <= 40
    assert _kkt(m, ipm, r.state) <= 1e-8
    assert ipm.cg_total <= 8 * r.iters


def test_hykkt_warm_start_removes_the_lifting_offset():
    """From the Lifted-KKT solution (E_0 <= 1e-8 of the lifted problem, about
    1e-5 from the original KKT point) a warm HyKKT solve lands on the reference
    point."""
    m = _column("small", 0)
    lip = LiftedIPM(m)
    rl = lip.solve(lip.cold_start(m.initial_guess(), 0.1), 0.1)
    assert rl.status == 0
    ref = ReferenceIPM(m).solve(m.initial_guess())
    off = np.max(np.abs(rl.state.y - ref.y))
    ipm = HyKKTIPM(m, IPMOptions(tol=1e-10, mu_min=1e-12))
    r = ipm.solve(ipm.from_lifted(rl.state), 1e-9)
    assert r.status == 0 and r.iters <= 12
    assert np.max(np.abs(r.state.y - ref.y)) <= 1e-7 < off
