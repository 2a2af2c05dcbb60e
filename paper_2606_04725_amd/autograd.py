"""torch.autograd.Function around one NMPC solve.

Forward runs nmpc_solve for the given parameters and returns the first-stage
control u_1* and the optimal objective f*; backward calls the sensitivity
entry point, which reuses the factorization of the condensed KKT matrix at the
solution (one forward/back solve with refinement per backward call).  The
handle holds one solution at a time: backward raises when the problem was
solved again, or its parameters changed, after the forward it belongs to.  With
CUDA tensors the parameters, u_1*, the seeds and the gradients stay on the GPU
(the *_dev entry points, ordered on torch's current stream); with CPU tensors
they cross the C ABI as host arrays.
"""
from __future__ import annotations

import numpy as np
import torch

from . import nmpc as N


def _host(t):
    return None if t is None else t.detach().to("cpu", torch.float64).numpy()


def _dev(t, device):
    return None if t is None else t.detach().to(device, torch.float64).contiguous()


def _ptr(t):
    return 0 if t is None else t.data_ptr()


class NMPCSolve(torch.autograd.Function):
    """u1, f = NMPCSolve.apply(problem, x0, setpoint, traj, u_prev, warm[, options])."""

    @staticmethod
    def forward(ctx, problem: N.Problem, x0, setpoint, traj, u_prev, warm: bool, options=None):
        cuda = x0.is_cuda
        dev = x0.device
        if cuda:
            stream = torch.cuda.current_stream(dev).cuda_stream
            xs = [_dev(t, dev) for t in (x0, setpoint, traj, u_prev)]
            problem.set_parameters_dev(*(_ptr(t) for t in xs), stream=stream)
        else:
            problem.set_parameters(_host(x0), setpoint=_host(setpoint), traj=_host(traj), u_prev=_host(u_prev))
        res = problem.solve(warm=bool(warm), options=options)
        if res.status != 0:
            raise N.NMPCError(res.status, f"solve ended with status {res.status}")
        if cuda:
            u1 = torch.empty(problem.nu, dtype=torch.float64, device=dev)
            problem.solution_dev(u1=u1.data_ptr(), stream=stream)
        else:
            u1 = torch.as_tensor(problem.first_stage()[0], dtype=torch.float64)
        ctx.problem = problem
        ctx.solution_id = problem.solution_id()[0]
        ctx.cuda = cuda
        ctx.device = dev
        ctx.shapes = (setpoint is not None, traj is not None, u_prev is not None)
        f = torch.tensor(res.objective, dtype=torch.float64, device=dev)
        return u1, f

    @staticmethod
    def backward(ctx, g_u1, g_f):
        p = ctx.problem
        sid, current = p.solution_id()
        if sid != ctx.solution_id or not current:
            # the handle holds another solution (a later solve or parameter
            # change on the same problem): its sensitivities are not this
            # forward's
            raise RuntimeError("NMPCSolve.backward: the problem was solved again or its parameters changed "
                               "after this forward; use one problem per differentiated solve")
        has_sp, has_tr, has_up = ctx.shapes
        dev = ctx.device
        if ctx.cuda:
            stream = torch.cuda.current_stream(dev).cuda_stream
            seed_u, seed_f = _dev(g_u1, dev), _dev(g_f, dev)
            e = lambda k: torch.empty(k, dtype=torch.float64, device=dev)  # noqa: E731
            gx, gs, gt, gu = e(p.nx), e(p.n_setpoint), e(p.n_traj), e(p.nu)
            p.adjoint_dev(_ptr(seed_u), _ptr(seed_f), gx.data_ptr(), gs.data_ptr(),
                          gt.data_ptr() if p.n_traj else 0, gu.data_ptr(), stream=stream)
            g = dict(x0=gx, setpoint=gs, traj=gt, u_prev=gu)
        else:
            seed = np.zeros(p.nu) if g_u1 is None else _host(g_u1)
            gobj = 0.0 if g_f is None else float(_host(g_f))
            _, gh = p.adjoint(seed, gobj)
            g = {k: torch.as_tensor(v, dtype=torch.float64, device=dev) for k, v in gh.items()}
        return (None, g["x0"], g["setpoint"] if has_sp else None, g["traj"] if has_tr else None,
                g["u_prev"] if has_up else None, None, None)
