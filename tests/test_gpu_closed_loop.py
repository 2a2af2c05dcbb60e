"""The closed loop on the device (nmpc_closed_loop_dev: Algorithm 1 with
plant = model, the parameter update and the first passes of each re-solve in
one captured graph) against the same loop driven from the host through
nmpc_set_parameters / nmpc_solve / nmpc_get_solution: the applied controls,
predicted states, iteration counts and the final iterate are identical bit for
bit, for several passes per graph; and the entry point's rules."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_04725_amd import capi
from paper_2606_04725_amd import nmpc as N
from plate_parity import note
from workloads import distillation_workload, reflux_workload

pytestmark = pytest.mark.gpu

STEPS = 8


def _column(w):
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    return p


def _host_loop(p, w, steps):
    us, xs, iters = [], [], 0
    for k in range(steps):
        u1, x1 = p.first_stage()
        us.append(u1)
        xs.append(x1)
        p.set_parameters(w.next_measurement(x1, k), setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(k + 1), u_prev=u1)
        r = p.solve(warm=True)
        assert r.status == 0
        iters += r.iters
    return np.array(us), np.array(xs), iters


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_device_loop_equals_host_loop(passes):
    import torch
    note(f"closed loop on the device vs host loop, small column, {STEPS} steps, {passes} passes per graph")
    w = distillation_workload("small", 0, n_resolves=STEPS + 1)
    ph, pd = _column(w), _column(w)
    assert ph.solve(warm=False).status == 0 and pd.solve(warm=False).status == 0
    us, xs, iters = _host_loop(ph, w, STEPS)
    dev = torch.device("cuda")
    traj = torch.tensor(np.array([w.zF(k + 1) for k in range(STEPS)]), dtype=torch.float64, device=dev)
    noise = torch.tensor(w.resolve_noise[:STEPS], dtype=torch.float64, device=dev)
    u_out = torch.zeros((STEPS, pd.nu), dtype=torch.float64, device=dev)
    x_out = torch.zeros((STEPS, pd.nx), dtype=torch.float64, device=dev)
    rc, done, it = pd.closed_loop_dev(STEPS, traj.data_ptr(), noise.data_ptr(), u_out.data_ptr(), x_out.data_ptr(),
                                      passes_per_step=passes)
    torch.cuda.synchronize()
    note(f"iterations host {iters} device {it}")
    assert rc == 0 and done == STEPS and it == iters
    assert np.array_equal(u_out.cpu().numpy(), us)
    assert np.array_equal(x_out.cpu().numpy(), xs)
    sh, sd = ph.solution(), pd.solution()
    for key in ("y", "lam", "omega_d", "zL", "zU"):
        assert np.array_equal(sh[key], sd[key]), key
    # the held solution is current for the loop's last parameters
    ident, current = pd.solution_id()
    assert current and ident == 1 + STEPS
    rc, _ = pd.adjoint(np.ones(pd.nu), 0.0)
    assert rc == 0


def test_device_loop_case_study():
    """The case study of Section 4.1 (plant = model, no noise, fixed setpoint)
    on the device for 30 steps equals the host loop."""
    note("closed loop on the device, case study, 30 steps")
    import torch
    w = reflux_workload()
    steps = 30

    def make():
        p = N.Problem(N.reflux_structure(w.H, dt=w.dt))
        p.analyze()
        p.set_parameters(w.x0, setpoint=[w.xbar, w.ubar], u_prev=[w.u_prev0])
        assert p.solve(warm=False).status == 0
        return p

    ph, pd = make(), make()
    us = []
    for k in range(steps):
        u1, x1 = ph.first_stage()
        us.append(u1)
        ph.set_parameters(x1, setpoint=[w.xbar, w.ubar], u_prev=u1)
        assert ph.solve(warm=True).status == 0
    u_out = torch.zeros((steps, 1), dtype=torch.float64, device="cuda")
    rc, done, _ = pd.closed_loop_dev(steps, u_out=u_out.data_ptr())
    torch.cuda.synchronize()
    assert rc == 0 and done == steps
    assert np.array_equal(u_out.cpu().numpy(), np.array(us))
    assert np.array_equal(ph.solution()["y"], pd.solution()["y"])


def test_device_loop_rules():
    note("closed loop on the device: rules")
    w = distillation_workload("small", 1)
    p = _column(w)
    with pytest.raises(N.NMPCError) as e:
        p.closed_loop_dev(2)                         # no solution held yet
    assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    assert p.solve(warm=False).status == 0
    with pytest.raises(N.NMPCError) as e:
        p.closed_loop_dev(2, options=N.default_options(timing=1))
    assert e.value.code == capi.NMPC_ERR_INVALID_ARG
    with pytest.raises(N.NMPCError) as e:
        p.closed_loop_dev(2, passes_per_step=0)
    assert e.value.code == capi.NMPC_ERR_INVALID_ARG
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    with pytest.raises(N.NMPCError) as e:
        p.closed_loop_dev(2)                         # parameters changed since the solve
    assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    assert p.solve(warm=False, options=N.default_options(kkt=capi.NMPC_KKT_HYKKT)).status == 0
    with pytest.raises(N.NMPCError) as e:
        p.closed_loop_dev(2)                         # a HyKKT iterate
    assert e.value.code == capi.NMPC_ERR_BAD_ORDER
    assert p.solve(warm=False).status == 0
    rc, done, it = p.closed_loop_dev(3)
    assert rc == 0 and done == 3 and it > 0
