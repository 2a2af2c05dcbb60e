"""Shared comparison of a GPU plate solve with the oracle's (test helper, not
collected).

Both sides solve with an E_0 tolerance that only the smallest barrier value
can meet from a cold start (PARITY_TOL), so they stop on the same barrier
problem.  Stopping there still leaves each iterate anywhere in the ball
E_mu <= PARITY_TOL around that problem's solution, and near an active bound the
ball is wide: a control at its lower bound sits at y = mu / z_L with
z_L ~ 5e-4, so a complementarity residual of 1e-9 moves y by ~2e-6.  Two
correct runs that stop one iteration apart therefore differ there by more
than 1e-6.  The comparison is made where the point is unique: each side takes
its own returned iterate into Newton's method on that one barrier problem
(fixed mu, the method's own step and line search) until E_mu <= TIGHT_TOL,
and the two tightened points are compared entry by entry.  The returned
points themselves are certified through the oracle's KKT evaluator and the
objective."""
import sys

import numpy as np

from oracle.kkt import kkt_error
from paper_2606_04725_amd import nmpc as N

# E_0 tolerance of the parity solves.  A cold start walks the barrier values
# 0.1, 0.02, 2.83e-3, 1.50e-4, 1.84e-6, 2.5e-9 and then mu_min = 1e-9; at
# 2.5e-9 the complementarity products s beta are about 2.5e-9, so E_0 cannot
# fall below 2e-9 there, while at mu_min it settles near 1e-9.
PARITY_TOL = 2e-9
# E_mu tolerance of the fixed-barrier tightening: the entries next to active
# bounds are then fixed to ~TIGHT_TOL / z_L ~ 2e-9
TIGHT_TOL = 1e-12


def note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def close(a, b, tol):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b))) / max(1.0, float(np.max(np.abs(b)))) <= tol


def rel_dev(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b))) / max(1.0, float(np.max(np.abs(b))))


def tighten_gpu(p, mu):
    """Newton's method on the barrier problem at ``mu`` from the handle's held
    iterate, on the GPU."""
    r = p.solve(warm=True, options=N.default_options(fixed_mu=1, tol=TIGHT_TOL, mu0_warm=mu, max_iter=30))
    assert r.status == 0, ("gpu tightening", r.status, r.iters)
    return r


def tighten_ref(ipm, res):
    """The same on the oracle, from its returned state."""
    t = ipm.solve(res.state, res.mu, fixed_mu=True, tol=TIGHT_TOL)
    assert t.status == 0, ("oracle tightening", t.status, t.iters)
    return t


def certify(m, ipm, sol, r, ref, iters_slack=2):
    """The returned points: both on mu_min, the original problem's KKT error
    <= 1e-8 by the oracle's evaluator, equal objective (1e-8), iteration counts
    within iters_slack (the filter's acceptance tests are threshold tests whose
    sums run in another order on the two sides, so a near-tie can cost one side
    an extra iteration on the way to the same barrier problem)."""
    note(f"iterations gpu {r.iters} oracle {ref.iters}; mu gpu {r.mu:.3e} oracle {ref.mu:.3e}")
    assert r.mu == ipm.o.mu_min and ref.mu == ipm.o.mu_min, (r.mu, ref.mu)
    e = kkt_error(m, sol["y"], sol["lam"], np.zeros(0), sol["zL"], sol["zU"])
    assert e["max"] <= 1e-8, e
    f_ref = m.f(ref.state.y)
    assert abs(m.f(sol["y"]) - f_ref) <= 1e-8 * max(1.0, abs(f_ref))
    assert abs(r.iters - ref.iters) <= iters_slack, (r.iters, ref.iters)


def compare_tight(m, sol, ref_t):
    """Tightened GPU point against the tightened oracle point: y, lambda, zL,
    zU within 1e-6 relative to max(1, |ref|) per block."""
    lam_ref = ref_t.state.omega[:m.m_c] - ref_t.state.omega[m.m_c:2 * m.m_c]
    for key, want in (("y", ref_t.state.y), ("lam", lam_ref), ("zL", ref_t.state.zL), ("zU", ref_t.state.zU)):
        d = rel_dev(sol[key], want)
        note(f"tightened {key}: {d:.2e}")
        assert d <= 1e-6, (key, d)


def solve_pair(m, p, ipm, ref, warm):
    """GPU solve (cold or warm from its held iterate) against the oracle result
    ``ref`` of the same start; returns the oracle's tightened result, from
    which the next warm re-solve of the oracle starts (the GPU's next one
    starts from its own tightened point)."""
    r = p.solve(warm=warm, options=N.default_options(tol=PARITY_TOL))
    assert r.status == 0, r.status
    certify(m, ipm, p.solution(), r, ref)
    tighten_gpu(p, r.mu)
    ref_t = tighten_ref(ipm, ref)
    compare_tight(m, p.solution(), ref_t)
    return ref_t
