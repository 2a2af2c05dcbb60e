"""The allocation-free Jacobian (nmpc_jacobian_u1_x0_noalloc) through the C ABI
against the allocating one (nmpc_jacobian_u1_x0) on the same solution: two
calls in a row share the GPU's fixed buffer, the second on a smaller problem,
then the first problem again (the buffer keeps the last call's contents, so
every value a call reads must be one it wrote)."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2606_04725_amd import capi
from paper_2606_04725_amd import nmpc as N
from workloads import distillation_workload, plate_workload

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _plate(G, H):
    w = plate_workload("large", 0, G=G, H=H)
    p = N.Problem(N.plate_structure(G, H, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
    p.analyze()
    p.set_parameters(w.T0, setpoint=w.target, u_prev=np.full(16, 0.5))
    assert p.solve().status == 0
    return p


def _column(kind, seed):
    w = distillation_workload(kind, seed, n_resolves=1)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    assert p.solve().status == 0
    return p


def _noalloc(p, torch):
    dev = torch.device("cuda:0")
    jac = torch.full((p.nu, p.nx), np.nan, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = capi.lib().nmpc_jacobian_u1_x0_noalloc(p._h, C.c_void_p(jac.data_ptr()), C.c_void_p(stream))
    torch.cuda.synchronize()
    return rc, jac.cpu().numpy()


def _check(p, torch, what):
    _note(f"noalloc jacobian: {what} (n {p.n}, nu {p.nu})")
    rc, J = _noalloc(p, torch)
    assert rc == 0, (rc, capi.lib().nmpc_last_error())
    rc2, Jref = p.jacobian_u1_x0()
    assert rc2 == 0
    dev = float(np.max(np.abs(J - Jref))) / max(1.0, float(np.max(np.abs(Jref))))
    _note(f"max relative deviation from the allocating entry point: {dev:.2e}")
    assert np.all(np.isfinite(J)) and dev <= 1e-12, dev


def test_noalloc_jacobian_matches_allocating_one():
    import torch
    big = _plate(16, 10)                      # large-front solves, 16 seeds
    _check(big, torch, "plate 16x16x10")
    small = _column("small", 2)               # second call: a smaller problem
    _check(small, torch, "distillation 10x20")
    medium = _column("medium", 0)
    _check(medium, torch, "distillation 40x100")
    _check(big, torch, "plate 16x16x10 again")


def test_noalloc_jacobian_refuses_stale_handle():
    import torch
    p = _column("small", 4)
    p.set_parameters(np.full(p.nx, 0.5))
    rc, _ = _noalloc(p, torch)
    assert rc == -2, rc   # NMPC_ERR_BAD_ORDER: parameters changed since the solve
