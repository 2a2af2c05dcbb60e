"""Receding-horizon loop on the oracle side, Algorithm 1.

Solve, extract the first control, apply it, take the next measurement, warm
start the next solve from the previous solution (unshifted as Algorithm 1
writes it, or shifted one stage) and update the parameters.  The plant is the transcription's own first stage: the predicted
x_1 is the implicit-Euler step of the model under u_1, to which the workload
adds its pre-drawn measurement noise.
"""
from __future__ import annotations

import time
import numpy as np

from .distillation import DistillationOCP
from .ipm import LiftedIPM, IPMOptions


def _shift_stages(v, stages, size):
    """Entries laid out stage by stage, ``size`` per stage: stage k takes stage
    k + 1's entries, the last stage keeps its own."""
    V = np.asarray(v).reshape(stages, size).copy()
    V[:-1] = V[1:]
    return V.reshape(-1)


def shift_state(m, st):
    """Shifted warm start of a Lifted-KKT iterate: every stage-indexed quantity
    moves one stage earlier (the solution predicted for stage k + 1 becomes the
    guess for stage k, since the horizon has advanced by one stage); the last
    stage keeps its values.  Lifted rows [plus | minus | inequality]: the
    stage-major equality rows move by their number per stage (rps: the state
    rows and, where the model has them, its algebraic rows; nx otherwise), the
    control-horizon hold rows (two per held stage) by two within the held
    stages, the inequality rows by two."""
    H, nx = m.H, m.nx
    rps = getattr(m, "rps", nx)
    dyn = H * rps
    held = (m.m_c - dyn) // 2          # held stages (two hold rows each)

    def rows(v):
        v = np.asarray(v)
        mc = m.m_c
        parts = []
        for blk in (v[:mc], v[mc:2 * mc]):
            parts.append(_shift_stages(blk[:dyn], H, rps))
            if held:
                parts.append(_shift_stages(blk[dyn:], held, 2))
        if m.m_d:
            parts.append(_shift_stages(v[2 * mc:], H, m.m_d // H))
        return np.concatenate(parts)

    return type(st)(_shift_stages(st.y, H, m.ns), rows(st.s), rows(st.omega), rows(st.beta),
                    _shift_stages(st.zL, H, m.ns), _shift_stages(st.zU, H, m.ns))


def distillation_episode(w, n_resolves=None, opts=None, record=False, shift=False):
    """Run one cold solve plus ``n_resolves`` warm re-solves of a distillation
    workload (each warm start shifted by one stage when ``shift``).  Returns a
    list of per-solve dicts (parameters in, solution out)."""
    n_resolves = w.n_resolves if n_resolves is None else n_resolves
    m = DistillationOCP.from_workload(w)
    ipm = LiftedIPM(m, opts or IPMOptions())
    x0, u_prev = w.x0.copy(), w.u_prev0.copy()
    out = []
    state = None
    for r in range(n_resolves + 1):
        zF = w.zF(r)
        m.set_parameters(x0=x0, zF=zF, u_prev=u_prev)
        t = time.perf_counter()
        if state is None:
            st0 = ipm.cold_start(m.initial_guess(), ipm.o.mu0_cold)
            res = ipm.solve(st0, ipm.o.mu0_cold, record=record)
        else:
            res = ipm.solve(shift_state(m, state) if shift else state, ipm.o.mu0_warm, record=record)
        dt = time.perf_counter() - t
        lam, om_d = ipm.multipliers(res.state)
        out.append(dict(index=r, x0=x0.copy(), zF=zF, u_prev=u_prev.copy(),
                        status=res.status, iters=res.iters, E0=res.E0, mu=res.mu,
                        y=res.state.y.copy(), lam=lam.copy(), omega_d=om_d.copy(),
                        zL=res.state.zL.copy(), zU=res.state.zU.copy(),
                        state=res.state.copy(), seconds=dt, trace=res.trace))
        state = res.state
        u_prev = m.u1(res.state.y)
        if r < n_resolves:
            x0 = w.next_measurement(m.x1(res.state.y), r)
    return m, out
