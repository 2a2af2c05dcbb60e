"""Python face of the C ABI: a thin handle wrapper around libnmpc.so.

All arithmetic runs inside the library (host symbolic analysis, HIP kernels for
everything numeric); this module only converts NumPy arrays to pointers and
status codes to exceptions.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import capi
from .capi import nmpc_options, nmpc_result, nmpc_structure


class NMPCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nmpc error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise NMPCError(rc, capi.lib().nmpc_last_error().decode())
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(capi._D)


def _ip(a):
    return None if a is None else a.ctypes.data_as(capi._I)


def _lp(a):
    return None if a is None else a.ctypes.data_as(capi._L)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def default_options(**over) -> nmpc_options:
    o = nmpc_options()
    capi.lib().nmpc_default_options(C.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o


def distillation_structure(N, H, dt, alpha, F=1.0, rho=1e-2, x_lo=0.0, x_hi=1.0, u_lo=0.5, u_hi=5.0,
                           ordering=capi.NMPC_ORDER_NESTED_DISSECTION, control_horizon=0):
    s = nmpc_structure()
    s.ordering = ordering
    s.control_horizon = control_horizon
    s.family = capi.NMPC_FAMILY_DISTILLATION
    s.horizon, s.dt, s.n_trays, s.alpha, s.feed_flow = H, dt, N, alpha, F
    s.move_penalty, s.x_lo, s.x_hi, s.u_lo, s.u_hi = rho, x_lo, x_hi, u_lo, u_hi
    return s


def reflux_structure(H, dt=2.0, N=32, Nf=17, D=0.2, F=0.4, alpha=1.6, xf=0.5, Ac=0.5, At=0.25, Ar=1.0, w_u=0.1,
                     u_lo=1.0, u_hi=5.0, flow_hi=10.0, ordering=capi.NMPC_ORDER_NESTED_DISSECTION):
    """The case-study column of Section 4.1 (defaults: Table 1)."""
    s = nmpc_structure()
    s.ordering = ordering
    s.family = capi.NMPC_FAMILY_REFLUX_COLUMN
    s.horizon, s.dt, s.n_trays, s.feed_tray, s.alpha, s.feed_flow = H, dt, N, Nf, alpha, F
    s.distillate, s.feed_comp, s.hold_cond, s.hold_tray, s.hold_reb = D, xf, Ac, At, Ar
    s.u_weight, s.x_lo, s.x_hi, s.u_lo, s.u_hi, s.flow_hi = w_u, 0.0, 1.0, u_lo, u_hi, flow_hi
    return s


def plate_structure(G, H, dt, cond_slope=0.1, t_hi=1.5, c_lo=0.0, c_hi=1.0,
                    ordering=capi.NMPC_ORDER_NESTED_DISSECTION):
    s = nmpc_structure()
    s.ordering = ordering
    s.family = capi.NMPC_FAMILY_HEATED_PLATE
    s.horizon, s.dt, s.grid = H, dt, G
    s.t_hi, s.c_lo, s.c_hi, s.cond_slope = t_hi, c_lo, c_hi, cond_slope
    return s


def stage_model_structure(gen, H, dt, ordering=capi.NMPC_ORDER_NESTED_DISSECTION):
    """Structure of a model compiled by the stage-pattern front end
    (simd.compile): its per-stage patterns, bounds and code object.  The
    arrays stay referenced by the returned structure until the problem is
    created (the library copies them then)."""
    if not gen.code:
        raise ValueError("the model has no code object (run simd.compile)")
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    keep = dict(row_ptr=i32(gen.row_ptr), row_cols=i32(gen.row_cols), prev_ptr=i32(gen.prev_ptr),
                prev_cols=i32(gen.prev_cols), prev_coef=_f64(gen.prev_coef), ineq_ptr=i32(gen.ineq_ptr),
                ineq_cols=i32(gen.ineq_cols), w_rows=i32(gen.w_rows), w_cols=i32(gen.w_cols),
                wx_rows=i32(gen.wx_rows), wx_cols=i32(gen.wx_cols), lb=_f64(gen.lb), ub=_f64(gen.ub),
                code=C.create_string_buffer(gen.code, len(gen.code)))
    d = capi.nmpc_stage_model()
    d.nx, d.nu, d.na, d.n_alg_rows = gen.nx, gen.nu, gen.na, gen.n_alg_rows
    d.n_setpoint, d.uses_traj = gen.n_setpoint, int(gen.uses_traj)
    for k in ("row_ptr", "row_cols", "prev_ptr", "prev_cols", "ineq_ptr", "ineq_cols", "w_rows", "w_cols",
              "wx_rows", "wx_cols"):
        setattr(d, k, _ip(keep[k]))
    for k in ("prev_coef", "lb", "ub"):
        setattr(d, k, _dp(keep[k]))
    d.n_ineq_rows = len(gen.ineq_ptr) - 1
    d.nw = len(gen.w_rows)
    d.nw_cross = len(gen.wx_rows)
    d.code_object = C.cast(keep["code"], C.c_void_p)
    d.code_object_size = len(gen.code)
    d.tag = gen.tag
    d.scratch_per_stage = int(gen.scratch_per_stage)
    s = nmpc_structure()
    s.ordering = ordering
    s.family = capi.NMPC_FAMILY_STAGE_MODEL
    s.horizon, s.dt = H, dt
    s.stage_model = C.pointer(d)
    s._keep = (keep, d)
    s._sizes = (gen.n_setpoint, H if gen.uses_traj else 0)
    return s


class Problem:
    """One transcribed OCP structure: create -> analyze -> set_parameters -> solve."""

    def __init__(self, structure: nmpc_structure):
        L = capi.lib()
        h = C.c_void_p()
        _check(L.nmpc_create_problem(C.byref(structure), C.byref(h)))
        self._h = h
        n, mc, md, nx, nu = (C.c_int32() for _ in range(5))
        nk = C.c_int64()
        _check(L.nmpc_sizes(h, C.byref(n), C.byref(mc), C.byref(md), C.byref(nx), C.byref(nu), C.byref(nk)))
        self.n, self.m_c, self.m_d, self.nx, self.nu = n.value, mc.value, md.value, nx.value, nu.value
        self.horizon = structure.horizon
        self.family = structure.family
        self._stage_sizes = getattr(structure, "_sizes", None)
        self.nnz_k = nk.value
        self.ml = 2 * self.m_c + self.m_d
        self.analyzed = False
        self.last_result = None

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().nmpc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- symbolic ------------------------------------------------------
    def analyze(self):
        _check(capi.lib().nmpc_analyze(self._h))
        self.analyzed = True

    def symbolic_sizes(self):
        ns, sl, nl, fl, rt, dp = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(capi.lib().nmpc_symbolic_sizes(self._h, C.byref(ns), C.byref(sl), C.byref(nl), C.byref(fl),
                                              C.byref(rt), C.byref(dp)))
        return dict(n_supernodes=ns.value, stored_l=sl.value, nnz_l=nl.value, flops=fl.value,
                    rows_total=rt.value, depth=dp.value)

    def export_symbolic(self):
        z = self.symbolic_sizes()
        n, ns = self.n, z["n_supernodes"]
        perm, parent, cc = (np.empty(n, np.int32) for _ in range(3))
        sp = np.empty(ns + 1, np.int32)
        rp = np.empty(ns + 1, np.int64)
        rows = np.empty(z["rows_total"], np.int32)
        _check(capi.lib().nmpc_export_symbolic(self._h, _ip(perm), _ip(parent), _ip(cc), _ip(sp), _lp(rp), _ip(rows)))
        return dict(perm=perm, parent=parent, colcount=cc, snode_ptr=sp, snode_rows_ptr=rp, snode_rows=rows, **z)

    def patterns(self):
        nj, nw, nk = C.c_int64(), C.c_int64(), C.c_int64()
        _check(capi.lib().nmpc_pattern_sizes(self._h, C.byref(nj), C.byref(nw), C.byref(nk)))
        jr, jc = np.empty(nj.value, np.int32), np.empty(nj.value, np.int32)
        wr, wc = np.empty(nw.value, np.int32), np.empty(nw.value, np.int32)
        kr = kc = None
        if self.analyzed:
            kr, kc = np.empty(nk.value, np.int32), np.empty(nk.value, np.int32)
        _check(capi.lib().nmpc_export_patterns(self._h, _ip(jr), _ip(jc), _ip(wr), _ip(wc), _ip(kr), _ip(kc)))
        return dict(j_rows=jr, j_cols=jc, w_rows=wr, w_cols=wc, k_rows=kr, k_cols=kc)

    # ---- parameters and solves -------------------------------------------
    def set_parameters(self, x0, setpoint=None, traj=None, u_prev=None):
        x0 = _f64(x0, self.nx)
        sp = None if setpoint is None else _f64(setpoint, self.n_setpoint)
        tr = None if traj is None else _f64(traj, self.horizon)
        up = None if u_prev is None else _f64(u_prev, self.nu)
        _check(capi.lib().nmpc_set_parameters(self._h, _dp(x0), _dp(sp), _dp(tr), _dp(up)))

    def solve(self, warm=False, options: nmpc_options | None = None) -> nmpc_result:
        r = nmpc_result()
        w = 2 if warm == "shift" else (1 if warm else 0)
        rc = capi.lib().nmpc_solve(self._h, w, None if options is None else C.byref(options),
                                   C.byref(r))
        _check(rc)
        self.last_result = r
        return r

    def first_stage(self):
        """(u1, x1) of the last solution: two small device-to-host copies."""
        u1, x1 = np.empty(self.nu), np.empty(self.nx)
        _check(capi.lib().nmpc_get_solution(self._h, None, None, None, None, None, _dp(u1), _dp(x1)))
        return u1, x1

    def solution(self):
        y, zl, zu = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        lam, om_d = np.empty(self.m_c), np.empty(max(self.m_d, 1))
        u1, x1 = np.empty(self.nu), np.empty(self.nx)
        _check(capi.lib().nmpc_get_solution(self._h, _dp(y), _dp(lam), _dp(om_d), _dp(zl), _dp(zu), _dp(u1),
                                            _dp(x1)))
        return dict(y=y, lam=lam, omega_d=om_d[:self.m_d], zL=zl, zU=zu, u1=u1, x1=x1)

    def get_iterate(self):
        n, ml = self.n, self.ml
        a = [np.empty(n), np.empty(ml), np.empty(ml), np.empty(ml), np.empty(n), np.empty(n)]
        _check(capi.lib().nmpc_get_iterate(self._h, *(_dp(v) for v in a)))
        return dict(zip(("y", "s", "omega", "beta", "zL", "zU"), a))

    def set_iterate(self, y, s, omega, beta, zL, zU):
        n, ml = self.n, self.ml
        a = [_f64(y, n), _f64(s, ml), _f64(omega, ml), _f64(beta, ml), _f64(zL, n), _f64(zU, n)]
        _check(capi.lib().nmpc_set_iterate(self._h, *(_dp(v) for v in a)))

    def autotune(self, reps=3):
        """Choose the front-kernel variant of every factor launch by timing;
        returns the number of launches that left the default variant."""
        ch = C.c_int32()
        _check(capi.lib().nmpc_autotune(self._h, int(reps), C.byref(ch)))
        return ch.value

    # ---- sensitivities ------------------------------------------------------
    def adjoint(self, seed_u1, seed_obj=0.0):
        """Vector-Jacobian product of seed_u1 . u1* + seed_obj f* with respect to
        the parameters; returns (status, dict of gradients).  Distillation:
        setpoint (xD*, xB*), traj zF[H]; plate: setpoint = target field, no traj."""
        gx, gs, gt, gu = np.empty(self.nx), np.empty(self.n_setpoint), np.empty(self.n_traj), np.empty(self.nu)
        rc = _check(capi.lib().nmpc_adjoint(self._h, _dp(_f64(seed_u1, self.nu)), float(seed_obj), _dp(gx),
                                            _dp(gs), _dp(gt), _dp(gu)))
        return rc, dict(x0=gx, setpoint=gs, traj=gt, u_prev=gu)

    # ---- device-pointer variants ----------------------------------------------
    # Addresses of float64 device buffers on the handle's GPU (0 = NULL) and the
    # caller's hipStream_t (0 = null stream); ordered on that stream, no host sync.
    @property
    def n_setpoint(self):
        if self.family == capi.NMPC_FAMILY_STAGE_MODEL:
            return self._stage_sizes[0]
        return self.nx if self.family == capi.NMPC_FAMILY_HEATED_PLATE else 2

    @property
    def n_traj(self):
        if self.family == capi.NMPC_FAMILY_STAGE_MODEL:
            return self._stage_sizes[1]
        return self.horizon if self.family == capi.NMPC_FAMILY_DISTILLATION else 0

    def set_parameters_dev(self, x0, setpoint=0, traj=0, u_prev=0, stream=0):
        _check(capi.lib().nmpc_set_parameters_dev(self._h, x0 or None, setpoint or None, traj or None,
                                                  u_prev or None, stream or None))

    def solution_dev(self, y=0, lam=0, omega_d=0, zL=0, zU=0, u1=0, x1=0, stream=0):
        _check(capi.lib().nmpc_get_solution_dev(self._h, y or None, lam or None, omega_d or None, zL or None,
                                                zU or None, u1 or None, x1 or None, stream or None))

    def adjoint_dev(self, seed_u1=0, seed_obj=0, grad_x0=0, grad_setpoint=0, grad_traj=0, grad_u_prev=0, stream=0):
        return _check(capi.lib().nmpc_adjoint_dev(self._h, seed_u1 or None, seed_obj or None, grad_x0 or None,
                                                  grad_setpoint or None, grad_traj or None, grad_u_prev or None,
                                                  stream or None))

    def closed_loop_dev(self, steps, traj=0, noise=0, u_out=0, x_out=0, passes_per_step=2,
                        options: nmpc_options | None = None, stream=0):
        """Device-resident closed loop (plant = model) from the held solution;
        device addresses (0 = NULL).  Returns (status, steps_done, iters)."""
        done, iters = C.c_int32(), C.c_int32()
        rc = _check(capi.lib().nmpc_closed_loop_dev(self._h, int(steps), traj or None, noise or None, u_out or None,
                                                    x_out or None, int(passes_per_step),
                                                    None if options is None else C.byref(options), C.byref(done),
                                                    C.byref(iters), stream or None))
        return rc, done.value, iters.value

    def solution_id(self):
        """(id, current): id counts the iterates the handle has taken; current is
        False once parameters were set after the last one."""
        i, c = C.c_int64(), C.c_int32()
        _check(capi.lib().nmpc_solution_id(self._h, C.byref(i), C.byref(c)))
        return i.value, bool(c.value)

    def jacobian_u1_x0(self):
        jac = np.empty((self.nu, self.nx))
        rc = _check(capi.lib().nmpc_jacobian_u1_x0(self._h, _dp(jac)))
        return rc, jac

    # ---- single steps -------------------------------------------------------
    def eval(self, y, lam, lam_d):
        z = self.pattern_counts()
        f = np.empty(1)
        g, c, d = np.empty(self.n), np.empty(self.m_c), np.empty(max(self.m_d, 1))
        jv, wv = np.empty(z[0]), np.empty(z[1])
        _check(capi.lib().nmpc_eval(self._h, _dp(_f64(y, self.n)), _dp(_f64(lam, self.m_c)),
                                    _dp(_f64(lam_d, self.m_d)), _dp(f), _dp(g), _dp(c), _dp(d), _dp(jv), _dp(wv)))
        return dict(f=float(f[0]), grad=g, c=c, d=d[:self.m_d], j_vals=jv, w_vals=wv)

    def pattern_counts(self):
        nj, nw, nk = C.c_int64(), C.c_int64(), C.c_int64()
        _check(capi.lib().nmpc_pattern_sizes(self._h, C.byref(nj), C.byref(nw), C.byref(nk)))
        return nj.value, nw.value, nk.value

    def factor(self, k_vals, eta=0.0, want_l=True):
        ok = C.c_int32()
        lv = np.empty(self.symbolic_sizes()["stored_l"]) if want_l else None
        _check(capi.lib().nmpc_factor(self._h, _dp(_f64(k_vals, self.nnz_k)), float(eta), C.byref(ok), _dp(lv)))
        return bool(ok.value), lv

    def linear_solve(self, b):
        x = np.empty(self.n)
        _check(capi.lib().nmpc_linear_solve(self._h, _dp(_f64(b, self.n)), _dp(x)))
        return x

    def assemble(self, mu):
        kv, rhs = np.empty(self.nnz_k), np.empty(self.n)
        _check(capi.lib().nmpc_assemble(self._h, float(mu), _dp(kv), _dp(rhs)))
        return kv, rhs


class Batch:
    """Several analyzed problems solved together (the batched form).  The batch
    references its problems; keep them alive while it exists."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[q._h.value for q in self.problems])
        h = C.c_void_p()
        _check(capi.lib().nmpc_batch_create(arr, len(self.problems), C.byref(h)))
        self._h = h

    def solve(self, warm=False, options: nmpc_options | None = None):
        """Returns (status, [nmpc_result per instance])."""
        res = (nmpc_result * len(self.problems))()
        rc = _check(capi.lib().nmpc_batch_solve(self._h, 2 if warm == "shift" else (1 if warm else 0),
                                                None if options is None else C.byref(options), res))
        return rc, list(res)

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().nmpc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_available() -> bool:
    return bool(capi.lib().nmpc_device_available())
