"""Device-pointer entry points (nmpc_*_dev) through the C ABI: the same solves,
solution and sensitivities as the host-array entry points, bit for bit, with
the data in torch CUDA tensors and the work ordered on torch's stream; and the
autograd function on CUDA tensors against the host path."""
import sys

import numpy as np
import pytest

from paper_2606_04725_amd import nmpc as N
from workloads import distillation_workload, plate_workload

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _column(seed=3):
    w = distillation_workload("small", seed, n_resolves=3)
    p = N.Problem(N.distillation_structure(w.N, w.H, w.dt, w.alpha, F=w.F, rho=w.rho))
    p.analyze()
    return w, p


def test_dev_entry_points_match_host_ones():
    import torch
    _note("set_parameters_dev / solution_dev / adjoint_dev vs host, distillation small")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    w, ph = _column()
    _, pd = _column()
    sp = [w.xD_sp, w.xB_sp]
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev)  # noqa: E731
    for k in range(2):
        x0 = w.x0 if k == 0 else w.next_measurement(ph.first_stage()[1], 0)
        ph.set_parameters(x0, setpoint=sp, traj=w.zF(k), u_prev=w.u_prev0)
        xt, st_, tt, ut = t(x0), t(sp), t(w.zF(k)), t(w.u_prev0)
        pd.set_parameters_dev(xt.data_ptr(), st_.data_ptr(), tt.data_ptr(), ut.data_ptr(), stream=stream)
        rh = ph.solve(warm=k > 0)
        rd = pd.solve(warm=k > 0)
        assert rh.status == 0 and rd.status == 0 and rh.iters == rd.iters
        sh = ph.solution()
        y, lam, zl, zu = (torch.empty(n, dtype=torch.float64, device=dev) for n in (pd.n, pd.m_c, pd.n, pd.n))
        om = torch.empty(max(pd.m_d, 1), dtype=torch.float64, device=dev)
        u1, x1 = torch.empty(pd.nu, dtype=torch.float64, device=dev), torch.empty(pd.nx, dtype=torch.float64, device=dev)
        pd.solution_dev(y.data_ptr(), lam.data_ptr(), om.data_ptr(), zl.data_ptr(), zu.data_ptr(), u1.data_ptr(),
                        x1.data_ptr(), stream=stream)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), sh["y"])
        assert np.array_equal(lam.cpu().numpy(), sh["lam"])
        assert np.array_equal(om.cpu().numpy()[:pd.m_d], sh["omega_d"])
        assert np.array_equal(zl.cpu().numpy(), sh["zL"]) and np.array_equal(zu.cpu().numpy(), sh["zU"])
        assert np.array_equal(u1.cpu().numpy(), sh["u1"]) and np.array_equal(x1.cpu().numpy(), sh["x1"])
        seed_u, seed_f = np.array([0.7, -1.3]), 0.25
        rc, gh = ph.adjoint(seed_u, seed_f)
        gx, gs, gt, gu = (torch.empty(n, dtype=torch.float64, device=dev) for n in (pd.nx, 2, pd.horizon, pd.nu))
        # the caller keeps its buffers alive until its stream has passed the call
        su_t, sf_t = t(seed_u), t([seed_f])
        rcd = pd.adjoint_dev(su_t.data_ptr(), sf_t.data_ptr(), gx.data_ptr(), gs.data_ptr(),
                             gt.data_ptr(), gu.data_ptr(), stream=stream)
        torch.cuda.synchronize()
        assert rc == rcd
        for key, v in (("x0", gx), ("setpoint", gs), ("traj", gt), ("u_prev", gu)):
            assert np.array_equal(v.cpu().numpy(), gh[key]), key


def test_dev_null_seeds_and_outputs():
    import torch
    _note("adjoint_dev with NULL seed_obj and outputs")
    dev = torch.device("cuda:0")
    w, p = _column(5)
    p.set_parameters(w.x0, setpoint=[w.xD_sp, w.xB_sp], traj=w.zF(0), u_prev=w.u_prev0)
    assert p.solve().status == 0
    _, gh = p.adjoint(np.array([1.0, 0.0]), 0.0)
    gx = torch.empty(p.nx, dtype=torch.float64, device=dev)
    seed = torch.tensor([1.0, 0.0], dtype=torch.float64, device=dev)
    p.adjoint_dev(seed.data_ptr(), 0, gx.data_ptr(), 0, 0, 0, stream=torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    assert np.array_equal(gx.cpu().numpy(), gh["x0"])


def test_dev_plate_adjoint_matches_host():
    import torch
    _note("plate 8x3 adjoint_dev vs host")
    dev = torch.device("cuda:0")
    w = plate_workload("large", 0, G=8, H=3)
    p = N.Problem(N.plate_structure(8, 3, w.dt, t_hi=w.T_hi, c_lo=w.u_lo, c_hi=w.u_hi))
    p.analyze()
    T0 = torch.tensor(w.T0, dtype=torch.float64, device=dev)
    tgt = torch.tensor(w.target, dtype=torch.float64, device=dev)
    up = torch.full((16,), 0.5, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    p.set_parameters_dev(T0.data_ptr(), tgt.data_ptr(), 0, up.data_ptr(), stream=stream)
    assert p.solve().status == 0
    rng = np.random.default_rng(3)
    su, so = rng.normal(size=16), float(rng.normal())
    rc, gh = p.adjoint(su, so)
    gx, gs, gu = (torch.empty(n, dtype=torch.float64, device=dev) for n in (64, 64, 16))
    su_t, so_t = torch.tensor(su, device=dev), torch.tensor([so], dtype=torch.float64, device=dev)
    p.adjoint_dev(su_t.data_ptr(), so_t.data_ptr(), gx.data_ptr(), gs.data_ptr(), 0, gu.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    assert np.array_equal(gx.cpu().numpy(), gh["x0"]) and np.array_equal(gs.cpu().numpy(), gh["setpoint"])


def test_autograd_on_cuda_tensors_matches_host_path():
    import torch
    from paper_2606_04725_amd.autograd import NMPCSolve
    _note("autograd with CUDA tensors vs CPU tensors")
    w, p = _column(2)
    out = {}
    for device in ("cpu", "cuda:0"):
        x0 = torch.tensor(w.x0, dtype=torch.float64, device=device, requires_grad=True)
        sp = torch.tensor([w.xD_sp, w.xB_sp], dtype=torch.float64, device=device, requires_grad=True)
        tr = torch.tensor(w.zF(0), dtype=torch.float64, device=device, requires_grad=True)
        up = torch.tensor(w.u_prev0, dtype=torch.float64, device=device)
        u1, f = NMPCSolve.apply(p, x0, sp, tr, up, False)
        loss = 2.0 * u1[0] - u1[1] + 0.5 * f
        loss.backward()
        assert u1.device == x0.device and x0.grad.device == x0.device
        out[device] = [t.detach().cpu().numpy() for t in (u1, f, x0.grad, sp.grad, tr.grad)]
    for a, b in zip(out["cpu"], out["cuda:0"]):
        assert np.array_equal(a, b)
