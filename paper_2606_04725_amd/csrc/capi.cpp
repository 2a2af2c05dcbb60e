// C ABI entry points: argument checks, error reporting, dispatch to the host
// symbolic phase and the device numeric phase.  No exception crosses the ABI.
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using nmpc::Problem;

struct nmpc_problem {
    Problem impl;
};

struct nmpc_batch {
    nmpc::Batch* impl = nullptr;
    std::vector<nmpc_problem*> members;
};

namespace {
thread_local std::string g_err;

nmpc_status fail(nmpc_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

bool all_finite(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

bool resolve_options(const nmpc_options* opts, nmpc_options& o) {
    nmpc_default_options(&o);
    if (opts) o = *opts;
    return o.tol > 0 && o.gamma > 0 && o.mu_min > 0 && o.max_iter >= 0 && o.ls_max >= 1 && o.mu0_cold > 0 &&
           o.mu0_warm > 0 && o.eta_first > 0 && o.kp_first > 1 && o.kp > 1 && o.eta_max > 0 && o.filter_cap >= 1 &&
           o.filter_cap <= nmpc::kFilterCapacity && o.alpha_min_frac > 0 &&
           o.soc_max >= 0 && o.soc_kappa > 0 &&
           (o.merit_fallback == 0 || o.merit_fallback == 1) && (o.fixed_mu == 0 || o.fixed_mu == 1) &&
           (o.kkt == NMPC_KKT_LIFTED || o.kkt == NMPC_KKT_HYKKT) && o.hykkt_gamma > 0 && o.hykkt_cg_tol > 0 &&
           o.hykkt_cg_max >= 1;
}

template <class F>
nmpc_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(NMPC_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(NMPC_ERR_INVALID_ARG, e.what());
    }
}
}  // namespace

extern "C" {

const char* nmpc_last_error(void) { return g_err.c_str(); }

nmpc_status nmpc_adjoint(nmpc_problem* p, const double* seed_u1, double seed_obj, double* grad_x0,
                         double* grad_setpoint, double* grad_traj, double* grad_uprev) {
    if (!p || !seed_u1) return fail(NMPC_ERR_INVALID_ARG, "adjoint: NULL handle or seed");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "adjoint: no solution yet");
    if (!p->impl.params_current) return fail(NMPC_ERR_BAD_ORDER, "adjoint: parameters changed since the last solve");
    if (p->impl.iter_hyk) return fail(NMPC_ERR_BAD_ORDER, "adjoint: the sensitivities need a Lifted-KKT solution");
    if (!std::isfinite(seed_obj) || !all_finite(seed_u1, p->impl.st.nu))
        return fail(NMPC_ERR_INVALID_ARG, "adjoint: non-finite seed");
    std::string err;
    nmpc_status rc = nmpc::device_adjoint(p->impl, seed_u1, seed_obj, grad_x0, grad_setpoint, grad_traj,
                                          grad_uprev, err);
    return rc >= 0 ? rc : fail(rc, err);
}

nmpc_status nmpc_jacobian_u1_x0(nmpc_problem* p, double* jac) {
    if (!p || !jac) return fail(NMPC_ERR_INVALID_ARG, "jacobian_u1_x0: NULL argument");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0: no solution yet");
    if (!p->impl.params_current)
        return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0: parameters changed since the last solve");
    if (p->impl.iter_hyk)
        return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0: the sensitivities need a Lifted-KKT solution");
    std::string err;
    nmpc_status rc = nmpc::device_jacobian_u1_x0(p->impl, jac, err);
    return rc >= 0 ? rc : fail(rc, err);
}

static_assert(nmpc::kNoAllocScratchBytes == NMPC_NOALLOC_SCRATCH_BYTES, "one size for the fixed buffer");

nmpc_status nmpc_jacobian_u1_x0_noalloc(nmpc_problem* p, double* jac, void* stream) {
    if (!p || !jac) return fail(NMPC_ERR_INVALID_ARG, "jacobian_u1_x0_noalloc: NULL argument");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0_noalloc: call nmpc_analyze first");
    const size_t need = nmpc::noalloc_scratch_bytes(p->impl);
    if (need > nmpc::kNoAllocScratchBytes)
        return fail(NMPC_ERR_UNSUPPORTED, "jacobian_u1_x0_noalloc: the problem needs " + std::to_string(need) +
                                              " bytes of scratch, more than the fixed " +
                                              std::to_string(nmpc::kNoAllocScratchBytes) +
                                              "; use nmpc_jacobian_u1_x0");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "jacobian_u1_x0_noalloc: no HIP device");
    if (!p->impl.have_iterate) return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0_noalloc: no solution yet");
    if (!p->impl.params_current)
        return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0_noalloc: parameters changed since the last solve");
    if (p->impl.iter_hyk)
        return fail(NMPC_ERR_BAD_ORDER, "jacobian_u1_x0_noalloc: the sensitivities need a Lifted-KKT solution");
    std::string err;
    nmpc_status rc = nmpc::device_jacobian_u1_x0_noalloc(p->impl, jac, stream, err);
    return rc >= 0 ? rc : fail(rc, err);
}

nmpc_status nmpc_set_parameters_dev(nmpc_problem* p, const double* x0, const double* setpoint, const double* traj,
                                    const double* u_prev, void* stream) {
    if (!p || !x0) return fail(NMPC_ERR_INVALID_ARG, "set_parameters_dev: NULL handle or x0");
    if (!p->impl.analyzed || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "set_parameters_dev: call nmpc_analyze first");
    nmpc::device_invalidate_adjoint(p->impl);
    p->impl.params_current = false;
    std::string err;
    nmpc_status rc = nmpc::device_set_parameters_dev(p->impl, x0, setpoint, traj, u_prev, stream, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_get_solution_dev(const nmpc_problem* p, double* y, double* lam, double* omega_d, double* zL,
                                  double* zU, double* u1, double* x1, void* stream) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "get_solution_dev: NULL handle");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "get_solution_dev: no solution yet");
    std::string err;
    nmpc_status rc = nmpc::device_get_solution_dev(p->impl, y, lam, omega_d, zL, zU, u1, x1, stream, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_adjoint_dev(nmpc_problem* p, const double* seed_u1, const double* seed_obj, double* grad_x0,
                             double* grad_setpoint, double* grad_traj, double* grad_uprev, void* stream) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "adjoint_dev: NULL handle");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "adjoint_dev: no solution yet");
    if (!p->impl.params_current) return fail(NMPC_ERR_BAD_ORDER, "adjoint_dev: parameters changed since the last solve");
    if (p->impl.iter_hyk) return fail(NMPC_ERR_BAD_ORDER, "adjoint_dev: the sensitivities need a Lifted-KKT solution");
    std::string err;
    nmpc_status rc = nmpc::device_adjoint_dev(p->impl, seed_u1, seed_obj, grad_x0, grad_setpoint, grad_traj,
                                              grad_uprev, stream, err);
    return rc >= 0 ? rc : fail(rc, err);
}

nmpc_status nmpc_autotune(nmpc_problem* p, int32_t reps, int32_t* changed) {
    if (!p || reps < 1) return fail(NMPC_ERR_INVALID_ARG, "autotune: NULL handle or reps < 1");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "autotune: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "autotune: no HIP device");
    return guarded([&]() -> nmpc_status {
        std::string err;
        int c = 0;
        nmpc_status rc = nmpc::device_autotune(p->impl, reps, &c, err);
        if (rc != NMPC_OK) return fail(rc, err);
        if (changed) *changed = c;
        return NMPC_OK;
    });
}

nmpc_status nmpc_solution_id(const nmpc_problem* p, int64_t* id, int32_t* current) {
    if (!p || !id) return fail(NMPC_ERR_INVALID_ARG, "solution_id: NULL argument");
    *id = p->impl.solution_id;
    if (current) *current = p->impl.params_current ? 1 : 0;
    return NMPC_OK;
}

int32_t nmpc_device_available(void) { return nmpc::device_present() ? 1 : 0; }

void nmpc_default_options(nmpc_options* o) {
    if (!o) return;
    o->tol = 1e-8;
    o->gamma = 1e-9;
    o->mu0_cold = 1e-1;
    o->mu0_warm = 1e-9;
    o->mu_min = 1e-9;
    o->kappa_eps = 10.0;
    o->kappa_mu = 0.2;
    o->theta_mu = 1.5;
    o->tau_min = 0.99;
    o->armijo = 1e-4;
    o->ls_max = 40;
    o->max_iter = 200;
    o->kappa_sigma = 1e10;
    o->eta_first = 1e-4;
    o->eta_min = 1e-20;
    o->eta_max = 1e40;
    o->kp_first = 100.0;
    o->kp = 8.0;
    o->km = 1.0 / 3.0;
    o->bound_push = 1e-2;
    o->slack_push = 1e-2;
    o->filter_gamma_theta = 1e-5;
    o->filter_gamma_phi = 1e-8;
    o->filter_s_theta = 1.1;
    o->filter_s_phi = 2.3;
    o->filter_delta = 1.0;
    o->alpha_min_frac = 0.05;
    o->theta_max_fact = 1e4;
    o->theta_min_fact = 1e-4;
    o->filter_cap = 128;
    o->soc_max = 4;
    o->soc_kappa = 0.99;
    o->merit_fallback = 1;
    o->timing = 0;
    o->graph = 1;
    o->fixed_mu = 0;
    o->kkt = NMPC_KKT_LIFTED;
    o->hykkt_gamma = 1e6;
    o->hykkt_cg_tol = 1e-12;
    o->hykkt_cg_max = 200;
}

nmpc_status nmpc_create_problem(const nmpc_structure* s, nmpc_problem** out) {
    if (!s || !out) return fail(NMPC_ERR_INVALID_ARG, "create_problem: NULL argument");
    *out = nullptr;
    return guarded([&]() -> nmpc_status {
        auto* h = new nmpc_problem();
        std::string err;
        if (!nmpc::build_structure(*s, h->impl.st, err)) {
            delete h;
            const bool known = s->family == NMPC_FAMILY_DISTILLATION || s->family == NMPC_FAMILY_HEATED_PLATE ||
                               s->family == NMPC_FAMILY_REFLUX_COLUMN || s->family == NMPC_FAMILY_STAGE_MODEL;
            return fail(known ? NMPC_ERR_INVALID_ARG : NMPC_ERR_UNSUPPORTED, err);
        }
        const auto& st = h->impl.st;
        h->impl.x0.assign(st.nx, 0.5);
        h->impl.setpoint.assign(2, 0.0);
        h->impl.traj.assign(st.H, 0.5);
        h->impl.u_prev.assign(st.nu, 0.0);
        if (s->family == NMPC_FAMILY_DISTILLATION) {
            h->impl.setpoint = {0.95, 0.05};
            h->impl.u_prev = {2.0, 2.5};
        } else if (s->family == NMPC_FAMILY_REFLUX_COLUMN) {   // the setpoint of Table 1, reflux ratio 2
            h->impl.setpoint = {0.8958, 2.51459};
            h->impl.u_prev = {2.0};
        } else if (s->family == NMPC_FAMILY_STAGE_MODEL) {   // zero parameters
            h->impl.x0.assign(st.nx, 0.0);
            h->impl.setpoint.assign(st.gm.nsp, 0.0);
            h->impl.traj.assign(st.H, 0.0);
        } else {                               // plate: zero field, zero target, mid-range heaters
            h->impl.x0.assign(st.nx, 0.0);
            h->impl.setpoint.assign(st.nx, 0.0);
            h->impl.u_prev.assign(st.nu, 0.5 * (s->c_lo + s->c_hi));
        }
        *out = h;
        return NMPC_OK;
    });
}

void nmpc_destroy(nmpc_problem* p) {
    if (!p) return;
    nmpc::device_free(p->impl);
    delete p;
}

nmpc_status nmpc_sizes(const nmpc_problem* p, int32_t* n, int32_t* m_c, int32_t* m_d, int32_t* nx,
                       int32_t* nu, int64_t* nnz_k) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "sizes: NULL handle");
    const auto& st = p->impl.st;
    if (n) *n = st.n;
    if (m_c) *m_c = st.m_c;
    if (m_d) *m_d = st.m_d;
    if (nx) *nx = st.nx;
    if (nu) *nu = st.nu;
    if (nnz_k) *nnz_k = st.nnz_k;
    return NMPC_OK;
}

nmpc_status nmpc_analyze(nmpc_problem* p) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "analyze: NULL handle");
    if (p->impl.analyzed) return NMPC_OK;
    return guarded([&]() -> nmpc_status {
        nmpc::symbolic_analyze(p->impl.st, p->impl.sym);
        p->impl.analyzed = true;
        if (nmpc::device_present()) {
            std::string err;
            nmpc_status rc = nmpc::device_init(p->impl, err);
            if (rc != NMPC_OK) return fail(rc, err);
        }
        return NMPC_OK;
    });
}

nmpc_status nmpc_symbolic_sizes(const nmpc_problem* p, int32_t* n_supernodes, int64_t* stored_l,
                                int64_t* nnz_l, int64_t* flops, int64_t* rows_total, int32_t* depth) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "symbolic_sizes: NULL handle");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "symbolic_sizes: call nmpc_analyze first");
    const auto& s = p->impl.sym;
    if (n_supernodes) *n_supernodes = s.nsn;
    if (stored_l) *stored_l = s.stored_l;
    if (nnz_l) *nnz_l = s.nnz_l;
    if (flops) *flops = s.flops;
    if (rows_total) *rows_total = (int64_t)s.sn_rows.size();
    if (depth) *depth = s.depth;
    return NMPC_OK;
}

nmpc_status nmpc_export_symbolic(const nmpc_problem* p, int32_t* perm, int32_t* parent, int32_t* colcount,
                                 int32_t* snode_ptr, int64_t* snode_rows_ptr, int32_t* snode_rows) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "export_symbolic: NULL handle");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "export_symbolic: call nmpc_analyze first");
    const auto& s = p->impl.sym;
    if (perm) std::memcpy(perm, s.perm.data(), s.perm.size() * sizeof(int32_t));
    if (parent) std::memcpy(parent, s.parent.data(), s.parent.size() * sizeof(int32_t));
    if (colcount) std::memcpy(colcount, s.colcount.data(), s.colcount.size() * sizeof(int32_t));
    if (snode_ptr) std::memcpy(snode_ptr, s.sn_ptr.data(), s.sn_ptr.size() * sizeof(int32_t));
    if (snode_rows_ptr) std::memcpy(snode_rows_ptr, s.sn_rows_ptr.data(), s.sn_rows_ptr.size() * sizeof(int64_t));
    if (snode_rows) std::memcpy(snode_rows, s.sn_rows.data(), s.sn_rows.size() * sizeof(int32_t));
    return NMPC_OK;
}

nmpc_status nmpc_pattern_sizes(const nmpc_problem* p, int64_t* nnz_j, int64_t* nnz_w, int64_t* nnz_k) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "pattern_sizes: NULL handle");
    const auto& st = p->impl.st;
    if (nnz_j) *nnz_j = (int64_t)st.jcol.size();
    if (nnz_w) *nnz_w = (int64_t)st.wrow.size();
    if (nnz_k) *nnz_k = st.nnz_k;
    return NMPC_OK;
}

nmpc_status nmpc_export_patterns(const nmpc_problem* p, int32_t* j_rows, int32_t* j_cols, int32_t* w_rows,
                                 int32_t* w_cols, int32_t* k_rows, int32_t* k_cols) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "export_patterns: NULL handle");
    const auto& st = p->impl.st;
    if (j_rows) std::memcpy(j_rows, st.jrow.data(), st.jrow.size() * sizeof(int32_t));
    if (j_cols) std::memcpy(j_cols, st.jcol.data(), st.jcol.size() * sizeof(int32_t));
    if (w_rows) std::memcpy(w_rows, st.wrow.data(), st.wrow.size() * sizeof(int32_t));
    if (w_cols) std::memcpy(w_cols, st.wcol.data(), st.wcol.size() * sizeof(int32_t));
    if (k_rows || k_cols) {
        if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "export_patterns: KKT slot order needs nmpc_analyze");
        const auto& s = p->impl.sym;
        if (k_rows) std::memcpy(k_rows, s.k_orow.data(), s.k_orow.size() * sizeof(int32_t));
        if (k_cols) std::memcpy(k_cols, s.k_ocol.data(), s.k_ocol.size() * sizeof(int32_t));
    }
    return NMPC_OK;
}

nmpc_status nmpc_set_parameters(nmpc_problem* p, const double* x0, const double* setpoint, const double* traj,
                                const double* u_prev) {
    if (!p || !x0) return fail(NMPC_ERR_INVALID_ARG, "set_parameters: NULL handle or x0");
    auto& P = p->impl;
    const auto& st = P.st;
    const size_t nsp = P.setpoint.size();
    if (!all_finite(x0, st.nx) || (setpoint && !all_finite(setpoint, nsp)) ||
        (traj && !all_finite(traj, st.H)) || (u_prev && !all_finite(u_prev, st.nu)))
        return fail(NMPC_ERR_INVALID_ARG, "set_parameters: non-finite value");
    P.x0.assign(x0, x0 + st.nx);
    if (setpoint) P.setpoint.assign(setpoint, setpoint + nsp);
    if (traj) P.traj.assign(traj, traj + st.H);
    if (u_prev) P.u_prev.assign(u_prev, u_prev + st.nu);
    P.params_current = false;
    if (P.dev) {
        nmpc::device_invalidate_adjoint(P);
        std::string err;
        nmpc_status rc = nmpc::device_set_parameters(P, err);
        if (rc != NMPC_OK) return fail(rc, err);
    }
    return NMPC_OK;
}

nmpc_status nmpc_solve(nmpc_problem* p, int32_t warm, const nmpc_options* opts, nmpc_result* res) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "solve: NULL handle");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "solve: call nmpc_analyze first");
    if (!nmpc::device_present() || !p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "solve: no HIP device");
    if (warm < 0 || warm > 2) return fail(NMPC_ERR_INVALID_ARG, "solve: warm must be 0, 1 or 2");
    if (warm && !p->impl.have_iterate) return fail(NMPC_ERR_BAD_ORDER, "solve: warm start without a previous iterate");
    nmpc_options o;
    if (!resolve_options(opts, o)) return fail(NMPC_ERR_INVALID_ARG, "solve: invalid options");
    if (warm && o.kkt == NMPC_KKT_LIFTED && p->impl.iter_hyk)
        return fail(NMPC_ERR_BAD_ORDER, "solve: a warm Lifted-KKT start needs a Lifted-KKT iterate (solve cold)");
    return guarded([&]() -> nmpc_status {
        nmpc_result r{};
        std::string err;
        auto t0 = std::chrono::steady_clock::now();
        nmpc_status rc = nmpc::device_solve(p->impl, warm, o, r, err);
        auto t1 = std::chrono::steady_clock::now();
        r.ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
        if (rc < 0) return fail(rc, err);
        p->impl.have_iterate = true;
        p->impl.params_current = true;
        p->impl.iter_hyk = o.kkt == NMPC_KKT_HYKKT;
        ++p->impl.solution_id;
        if (res) *res = r;
        return rc;
    });
}

nmpc_status nmpc_closed_loop_dev(nmpc_problem* p, int32_t steps, const double* traj, const double* noise,
                                 double* u_out, double* x_out, int32_t passes_per_step, const nmpc_options* opts,
                                 int32_t* steps_done, int32_t* iters_total, void* stream) {
    if (!p || !steps_done || !iters_total) return fail(NMPC_ERR_INVALID_ARG, "closed_loop: NULL argument");
    *steps_done = 0;
    *iters_total = 0;
    if (steps < 0 || passes_per_step < 1 || passes_per_step > 16)
        return fail(NMPC_ERR_INVALID_ARG, "closed_loop: need steps >= 0 and 1 <= passes_per_step <= 16");
    if (!p->impl.analyzed || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "closed_loop: call nmpc_analyze first");
    if (!p->impl.have_iterate || !p->impl.params_current || p->impl.iter_hyk)
        return fail(NMPC_ERR_BAD_ORDER, "closed_loop: needs a Lifted-KKT solution for the current parameters");
    nmpc_options o;
    if (!resolve_options(opts, o)) return fail(NMPC_ERR_INVALID_ARG, "closed_loop: invalid options");
    if (o.kkt != NMPC_KKT_LIFTED || o.timing != 0)
        return fail(NMPC_ERR_INVALID_ARG, "closed_loop: needs kkt = NMPC_KKT_LIFTED and timing = 0");
    if (steps == 0) return NMPC_OK;
    return guarded([&]() -> nmpc_status {
        std::string err;
        int done = 0, iters = 0;
        nmpc_status rc = nmpc::device_closed_loop(p->impl, steps, traj, noise, u_out, x_out, passes_per_step, o,
                                                  stream, &done, &iters, err);
        *steps_done = done;
        *iters_total = iters;
        if (rc < 0) return fail(rc, err);
        p->impl.have_iterate = true;
        p->impl.params_current = true;
        p->impl.iter_hyk = false;
        p->impl.solution_id += done;
        return rc;
    });
}

nmpc_status nmpc_get_solution(const nmpc_problem* p, double* y, double* lam, double* omega_d, double* zL,
                              double* zU, double* u1, double* x1) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "get_solution: NULL handle");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "get_solution: no solution yet");
    if (!y && !lam && !omega_d && !zL && !zU) {   // first-stage values only: two small copies
        std::string err;
        nmpc_status rc = nmpc::device_get_first_stage(p->impl, u1, x1, err);
        return rc == NMPC_OK ? rc : fail(rc, err);
    }
    return guarded([&]() -> nmpc_status {
        const auto& st = p->impl.st;
        const int ml = 2 * st.m_c + st.m_d;
        std::vector<double> Y(st.n), S(ml), Om(ml), B(ml), ZL(st.n), ZU(st.n);
        std::string err;
        nmpc_status rc = nmpc::device_get_iterate(p->impl, Y.data(), S.data(), Om.data(), B.data(), ZL.data(),
                                                  ZU.data(), err);
        if (rc != NMPC_OK) return fail(rc, err);
        if (y) std::memcpy(y, Y.data(), st.n * sizeof(double));
        if (lam)
            for (int r = 0; r < st.m_c; ++r) lam[r] = Om[r] - Om[st.m_c + r];
        if (omega_d)
            for (int r = 0; r < st.m_d; ++r) omega_d[r] = Om[2 * st.m_c + r];
        if (zL) std::memcpy(zL, ZL.data(), st.n * sizeof(double));
        if (zU) std::memcpy(zU, ZU.data(), st.n * sizeof(double));
        const int ns = st.n / st.H;
        if (u1)
            for (int j = 0; j < st.nu; ++j) u1[j] = Y[st.nx + j];
        if (x1)
            for (int j = 0; j < st.nx; ++j) x1[j] = Y[j];
        (void)ns;
        return NMPC_OK;
    });
}

nmpc_status nmpc_get_iterate(const nmpc_problem* p, double* y, double* s, double* omega, double* beta, double* zL,
                             double* zU) {
    if (!p || !y || !s || !omega || !beta || !zL || !zU) return fail(NMPC_ERR_INVALID_ARG, "get_iterate: NULL argument");
    if (!p->impl.have_iterate || !p->impl.dev) return fail(NMPC_ERR_BAD_ORDER, "get_iterate: no iterate yet");
    std::string err;
    nmpc_status rc = nmpc::device_get_iterate(p->impl, y, s, omega, beta, zL, zU, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_set_iterate(nmpc_problem* p, const double* y, const double* s, const double* omega,
                             const double* beta, const double* zL, const double* zU) {
    if (!p || !y || !s || !omega || !beta || !zL || !zU) return fail(NMPC_ERR_INVALID_ARG, "set_iterate: NULL argument");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "set_iterate: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "set_iterate: no HIP device");
    const auto& st = p->impl.st;
    const size_t ml = 2 * st.m_c + st.m_d;
    if (!all_finite(y, st.n) || !all_finite(s, ml) || !all_finite(omega, ml) || !all_finite(beta, ml) ||
        !all_finite(zL, st.n) || !all_finite(zU, st.n))
        return fail(NMPC_ERR_INVALID_ARG, "set_iterate: non-finite value");
    for (size_t i = 0; i < ml; ++i)
        if (!(s[i] > 0) || !(beta[i] > 0)) return fail(NMPC_ERR_INVALID_ARG, "set_iterate: s and beta must be > 0");
    std::string err;
    nmpc_status rc = nmpc::device_set_iterate(p->impl, y, s, omega, beta, zL, zU, err);
    if (rc != NMPC_OK) return fail(rc, err);
    p->impl.have_iterate = true;
    p->impl.params_current = true;
    p->impl.iter_hyk = false;
    ++p->impl.solution_id;
    return NMPC_OK;
}

nmpc_status nmpc_eval(nmpc_problem* p, const double* y, const double* lam, const double* lam_d, double* f,
                      double* grad, double* c, double* d, double* j_vals, double* w_vals) {
    if (!p || !y || !lam || (!lam_d && p->impl.st.m_d)) return fail(NMPC_ERR_INVALID_ARG, "eval: NULL argument");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "eval: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "eval: no HIP device");
    std::string err;
    nmpc_status rc = nmpc::device_eval(p->impl, y, lam, lam_d, f, grad, c, d, j_vals, w_vals, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_factor(nmpc_problem* p, const double* k_vals, double eta, int32_t* ok, double* l_vals) {
    if (!p || !k_vals || !ok) return fail(NMPC_ERR_INVALID_ARG, "factor: NULL argument");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "factor: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "factor: no HIP device");
    if (!std::isfinite(eta) || eta < 0) return fail(NMPC_ERR_INVALID_ARG, "factor: eta must be finite and >= 0");
    std::string err;
    nmpc_status rc = nmpc::device_factor(p->impl, k_vals, eta, ok, l_vals, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_linear_solve(nmpc_problem* p, const double* b, double* x) {
    if (!p || !b || !x) return fail(NMPC_ERR_INVALID_ARG, "linear_solve: NULL argument");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "linear_solve: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "linear_solve: no HIP device");
    std::string err;
    nmpc_status rc = nmpc::device_linear_solve(p->impl, b, x, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_assemble(nmpc_problem* p, double mu, double* k_vals, double* rhs) {
    if (!p) return fail(NMPC_ERR_INVALID_ARG, "assemble: NULL handle");
    if (!p->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "assemble: call nmpc_analyze first");
    if (!p->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "assemble: no HIP device");
    if (!p->impl.have_iterate) return fail(NMPC_ERR_BAD_ORDER, "assemble: no iterate (solve or set_iterate first)");
    if (!(mu > 0)) return fail(NMPC_ERR_INVALID_ARG, "assemble: mu must be > 0");
    std::string err;
    nmpc_status rc = nmpc::device_assemble(p->impl, mu, k_vals, rhs, err);
    return rc == NMPC_OK ? rc : fail(rc, err);
}

nmpc_status nmpc_batch_create(nmpc_problem* const* problems, int32_t count, nmpc_batch** out) {
    if (!problems || !out || count < 1) return fail(NMPC_ERR_INVALID_ARG, "batch_create: NULL argument or count < 1");
    *out = nullptr;
    for (int32_t i = 0; i < count; ++i) {
        if (!problems[i]) return fail(NMPC_ERR_INVALID_ARG, "batch_create: NULL problem");
        for (int32_t j = 0; j < i; ++j)
            if (problems[j] == problems[i]) return fail(NMPC_ERR_INVALID_ARG, "batch_create: a problem appears twice");
    }
    std::vector<Problem*> ps;
    for (int32_t i = 0; i < count; ++i) {
        nmpc_problem* q = problems[i];
        if (!q->impl.analyzed) return fail(NMPC_ERR_BAD_ORDER, "batch_create: every problem must be analyzed");
        if (!q->impl.dev) return fail(NMPC_ERR_NO_DEVICE, "batch_create: no HIP device");
        ps.push_back(&q->impl);
    }
    return guarded([&]() -> nmpc_status {
        auto* b = new nmpc_batch();
        std::string err;
        nmpc_status rc = nmpc::batch_create(ps, b->impl, err);
        if (rc != NMPC_OK) {
            delete b;
            return fail(rc, err);
        }
        b->members.assign(problems, problems + count);
        *out = b;
        return NMPC_OK;
    });
}

nmpc_status nmpc_batch_solve(nmpc_batch* b, int32_t warm, const nmpc_options* opts, nmpc_result* per_instance) {
    if (!b || !b->impl) return fail(NMPC_ERR_INVALID_ARG, "batch_solve: NULL batch");
    if (warm < 0 || warm > 2) return fail(NMPC_ERR_INVALID_ARG, "batch_solve: warm must be 0, 1 or 2");
    if (warm)
        for (auto* q : b->members)
            if (!q->impl.have_iterate)
                return fail(NMPC_ERR_BAD_ORDER, "batch_solve: warm start without a previous iterate");
    nmpc_options o;
    if (!resolve_options(opts, o)) return fail(NMPC_ERR_INVALID_ARG, "batch_solve: invalid options");
    if (o.kkt != NMPC_KKT_LIFTED) return fail(NMPC_ERR_UNSUPPORTED, "batch_solve: HyKKT solves one problem at a time");
    if (warm)
        for (auto* q : b->members)
            if (q->impl.iter_hyk)
                return fail(NMPC_ERR_BAD_ORDER, "batch_solve: a warm Lifted-KKT start needs a Lifted-KKT iterate");
    return guarded([&]() -> nmpc_status {
        std::vector<nmpc_result> r(b->members.size());
        std::string err;
        auto t0 = std::chrono::steady_clock::now();
        nmpc_status rc = nmpc::batch_solve(*b->impl, warm, o, r.data(), err);
        auto t1 = std::chrono::steady_clock::now();
        if (rc < 0) return fail(rc, err);
        const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        for (size_t i = 0; i < r.size(); ++i) {
            r[i].ms_total = ms;
            b->members[i]->impl.have_iterate = true;
            b->members[i]->impl.params_current = true;
            b->members[i]->impl.iter_hyk = false;
            ++b->members[i]->impl.solution_id;
            nmpc::device_invalidate_adjoint(b->members[i]->impl);
        }
        if (per_instance) std::copy(r.begin(), r.end(), per_instance);
        return rc;
    });
}

void nmpc_batch_destroy(nmpc_batch* b) {
    if (!b) return;
    nmpc::batch_free(b->impl);
    delete b;
}

}  // extern "C"
