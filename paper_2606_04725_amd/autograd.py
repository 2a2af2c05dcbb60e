"""torch.autograd.Function around one NMPC solve.

Forward runs nmpc_solve for the given parameters and returns the first-stage
control u_1* and the optimal objective f*; backward calls nmpc_adjoint, which
reuses the factorization of the condensed KKT matrix at the solution (one
forward/back solve per backward call).  Parameter vectors are tiny, so they
cross the C ABI as host arrays.
"""
from __future__ import annotations

import numpy as np
import torch

from . import nmpc as N


def _host(t):
    return None if t is None else t.detach().to("cpu", torch.float64).numpy()


class NMPCSolve(torch.autograd.Function):
    """u1, f = NMPCSolve.apply(problem, x0, setpoint, traj, u_prev, warm)."""

    @staticmethod
    def forward(ctx, problem: N.Problem, x0, setpoint, traj, u_prev, warm: bool):
        problem.set_parameters(_host(x0), setpoint=_host(setpoint), traj=_host(traj), u_prev=_host(u_prev))
        res = problem.solve(warm=bool(warm))
        if res.status != 0:
            raise N.NMPCError(res.status, f"solve ended with status {res.status}")
        sol = problem.solution()
        ctx.problem = problem
        ctx.device = x0.device
        ctx.shapes = (setpoint is not None, traj is not None, u_prev is not None)
        u1 = torch.as_tensor(sol["u1"], dtype=torch.float64, device=x0.device)
        f = torch.tensor(res.objective, dtype=torch.float64, device=x0.device)
        return u1, f

    @staticmethod
    def backward(ctx, g_u1, g_f):
        p = ctx.problem
        seed = np.zeros(p.nu) if g_u1 is None else _host(g_u1)
        gobj = 0.0 if g_f is None else float(_host(g_f))
        _, g = p.adjoint(seed, gobj)
        dev = ctx.device
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)  # noqa: E731
        has_sp, has_tr, has_up = ctx.shapes
        return (None, t(g["x0"]), t(g["setpoint"]) if has_sp else None, t(g["traj"]) if has_tr else None,
                t(g["u_prev"]) if has_up else None, None)
