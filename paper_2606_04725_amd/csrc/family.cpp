// Direct transcription of the supported OCP families into fixed sparsity
// patterns (Section 3.1, eqs. 5-6).  Only structure is built here; numeric
// values come from the device eval kernels.
#include <algorithm>
#include <cmath>

#include "distill_layout.h"
#include "plate_layout.h"
#include "reflux_layout.h"
#include "internal.h"

namespace nmpc {

static void finish_k_count(Structure& st) {
    // nnz of the lower pattern of W + J^T J + diag (structural union)
    std::vector<int64_t> keys;
    const int64_t n = st.n;
    keys.reserve(st.wrow.size() + 8 * st.jcol.size() + st.n);
    for (size_t e = 0; e < st.wrow.size(); ++e) {
        int64_t a = std::max(st.wrow[e], st.wcol[e]), b = std::min(st.wrow[e], st.wcol[e]);
        keys.push_back(a * n + b);
    }
    const int m = st.m_c + st.m_d;
    for (int r = 0; r < m; ++r) {
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p)
            for (int q = st.jptr[r]; q <= p; ++q) {
                int64_t a = std::max(st.jcol[p], st.jcol[q]), b = std::min(st.jcol[p], st.jcol[q]);
                keys.push_back(a * n + b);
            }
    }
    for (int64_t j = 0; j < n; ++j) keys.push_back(j * n + j);
    std::sort(keys.begin(), keys.end());
    st.nnz_k = std::unique(keys.begin(), keys.end()) - keys.begin();
}

static bool build_distillation(const nmpc_structure& s, Structure& st, std::string& err) {
    if (s.n_trays < 2 || s.horizon < 1 || !(s.dt > 0) || !(s.alpha > 1.0) || !(s.feed_flow >= 0) ||
        !(s.x_lo < s.x_hi) || !(s.u_lo < s.u_hi) || !(s.move_penalty >= 0) || s.control_horizon < 0) {
        err = "distillation: need n_trays >= 2, horizon >= 1, dt > 0, alpha > 1, valid bounds, control_horizon >= 0";
        return false;
    }
    DistillDims D;
    D.N = s.n_trays;
    D.nx = D.N + 2;
    D.ns = D.nx + 2;
    D.H = s.horizon;
    D.fd = D.N / 2;
    D.hc = (s.control_horizon >= 1 && s.control_horizon < s.horizon) ? s.control_horizon : s.horizon;
    st.nx = D.nx;
    st.nu = 2;
    st.H = D.H;
    st.n = D.H * D.ns;
    st.m_c = D.H * D.nx + 2 * (D.H - D.hc);
    st.m_d = 2 * D.H;
    const int m = st.m_c + st.m_d;
    st.jptr.assign(m + 1, 0);
    st.jcol.clear();
    st.jrow.clear();
    for (int k = 0; k < D.H; ++k)
        for (int i = 0; i < D.nx; ++i) {
            const int row = k * D.nx + i;
            const int base = k * D.ns;
            if (k > 0) st.jcol.push_back((k - 1) * D.ns + i);
            if (i > 0) st.jcol.push_back(base + i - 1);
            st.jcol.push_back(base + i);
            if (i < D.nx - 1) st.jcol.push_back(base + i + 1);
            if (i > 0) st.jcol.push_back(base + D.nx);
            st.jcol.push_back(base + D.nx + 1);
            st.jptr[row + 1] = (int)st.jcol.size();
            if (st.jptr[row + 1] - st.jptr[row] != dl_row_nnz(D, k, i)) {
                err = "internal: distillation row layout mismatch";
                return false;
            }
        }
    for (int k = D.hc; k < D.H; ++k)     // control-horizon holds u_k - u_{k-1}
        for (int j = 0; j < 2; ++j) {
            st.jcol.push_back((k - 1) * D.ns + D.nx + j);
            st.jcol.push_back(k * D.ns + D.nx + j);
            st.jptr[D.H * D.nx + 2 * (k - D.hc) + j + 1] = (int)st.jcol.size();
        }
    for (int k = 0; k < D.H; ++k)
        for (int r = 0; r < 2; ++r) {
            st.jcol.push_back(k * D.ns + D.nx);
            st.jcol.push_back(k * D.ns + D.nx + 1);
            st.jptr[st.m_c + 2 * k + r + 1] = (int)st.jcol.size();
        }
    st.jrow.resize(st.jcol.size());
    for (int r = 0; r < m; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p) st.jrow[p] = r;
    // lower Hessian slots in the kernel's order
    const int nw = dl_nnz_w(D);
    st.wrow.assign(nw, 0);
    st.wcol.assign(nw, 0);
    for (int k = 0; k < D.H; ++k) {
        const int o = k * dl_wstage(D), b = k * D.ns, iR = b + D.nx, iV = b + D.nx + 1;
        for (int i = 0; i < D.nx; ++i) {
            st.wrow[o + i] = b + i;            st.wcol[o + i] = b + i;
            st.wrow[o + D.nx + i] = iR;        st.wcol[o + D.nx + i] = b + i;
            st.wrow[o + 2 * D.nx + 1 + i] = iV; st.wcol[o + 2 * D.nx + 1 + i] = b + i;
        }
        st.wrow[o + 2 * D.nx] = iR;     st.wcol[o + 2 * D.nx] = iR;
        st.wrow[o + 3 * D.nx + 1] = iV; st.wcol[o + 3 * D.nx + 1] = iV;
        if (k > 0) {
            const int c = dl_wcross(D, k);
            st.wrow[c] = iR;     st.wcol[c] = iR - D.ns;
            st.wrow[c + 1] = iV; st.wcol[c + 1] = iV - D.ns;
        }
    }
    st.lb.assign(st.n, 0.0);
    st.ub.assign(st.n, 0.0);
    for (int k = 0; k < D.H; ++k)
        for (int j = 0; j < D.ns; ++j) {
            const bool is_x = j < D.nx;
            st.lb[k * D.ns + j] = is_x ? s.x_lo : s.u_lo;
            st.ub[k * D.ns + j] = is_x ? s.x_hi : s.u_hi;
        }
    return true;
}

static bool build_plate(const nmpc_structure& s, Structure& st, std::string& err) {
    if (s.grid < 4 || s.grid % 4 != 0 || s.horizon < 1 || !(s.dt > 0) || !(s.c_lo < s.c_hi) ||
        !(s.cond_slope >= 0) || !(s.t_hi > -INFINITY) || s.control_horizon != 0) {
        err = "plate: need grid a positive multiple of 4, horizon >= 1, dt > 0, c_lo < c_hi, cond_slope >= 0, "
              "control_horizon 0";
        return false;
    }
    PlateDims D;
    D.G = s.grid;
    D.nx = D.G * D.G;
    D.ns = D.nx + 16;
    D.H = s.horizon;
    D.q = D.G / 4;
    st.nx = D.nx;
    st.nu = 16;
    st.H = D.H;
    st.n = D.H * D.ns;
    st.m_c = D.H * D.nx;
    st.m_d = 0;
    st.jptr.assign(st.m_c + 1, 0);
    st.jcol.clear();
    for (int k = 0; k < D.H; ++k)
        for (int p = 0; p < D.nx; ++p) {
            const int b = p / D.G, a = p - b * D.G, base = k * D.ns;
            if (k > 0) st.jcol.push_back((k - 1) * D.ns + p);
            if (b > 0) st.jcol.push_back(base + p - D.G);
            if (a > 0) st.jcol.push_back(base + p - 1);
            st.jcol.push_back(base + p);
            if (a < D.G - 1) st.jcol.push_back(base + p + 1);
            if (b < D.G - 1) st.jcol.push_back(base + p + D.G);
            if (b == 0) st.jcol.push_back(base + D.nx + 0 * 4 + a / D.q);
            if (a == D.G - 1) st.jcol.push_back(base + D.nx + 1 * 4 + b / D.q);
            if (b == D.G - 1) st.jcol.push_back(base + D.nx + 2 * 4 + a / D.q);
            if (a == 0) st.jcol.push_back(base + D.nx + 3 * 4 + b / D.q);
            const int row = k * D.nx + p;
            st.jptr[row + 1] = (int)st.jcol.size();
            if (st.jptr[row + 1] - st.jptr[row] != pl_row_nnz(D, k, p)) {
                err = "internal: plate row layout mismatch";
                return false;
            }
        }
    st.jrow.resize(st.jcol.size());
    for (int r = 0; r < st.m_c; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p) st.jrow[p] = r;
    st.wrow.resize(st.n);
    st.wcol.resize(st.n);
    for (int j = 0; j < st.n; ++j) st.wrow[j] = st.wcol[j] = j;
    st.lb.assign(st.n, 0.0);
    st.ub.assign(st.n, 0.0);
    for (int k = 0; k < D.H; ++k)
        for (int j = 0; j < D.ns; ++j) {
            const bool is_t = j < D.nx;
            st.lb[k * D.ns + j] = is_t ? -INFINITY : s.c_lo;
            st.ub[k * D.ns + j] = is_t ? s.t_hi : s.c_hi;
        }
    return true;
}

static bool build_reflux(const nmpc_structure& s, Structure& st, std::string& err) {
    if (s.n_trays < 4 || s.feed_tray < 2 || s.feed_tray > s.n_trays - 2 || s.horizon < 1 || !(s.dt > 0) ||
        !(s.alpha > 1.0) || !(s.feed_flow > 0) || !(s.distillate > 0) || !(s.distillate < s.feed_flow) ||
        !(s.hold_cond > 0) || !(s.hold_tray > 0) || !(s.hold_reb > 0) || !(s.u_weight >= 0) ||
        !(s.x_lo < s.x_hi) || !(s.u_lo < s.u_hi) || !(s.flow_hi > 0) || s.control_horizon != 0) {
        err = "reflux column: need n_trays >= 4, 2 <= feed_tray <= n_trays - 2, horizon >= 1, dt > 0, alpha > 1, "
              "0 < distillate < feed_flow, positive holdups, u_weight >= 0, valid bounds, control_horizon 0";
        return false;
    }
    RefluxDims D{s.n_trays, s.feed_tray, 2 * s.n_trays + 4, 2 * s.n_trays + 3, s.horizon};
    const int N = D.N;
    st.nx = N;
    st.nu = 1;
    st.H = D.H;
    st.n = D.H * D.ns;
    st.m_c = D.H * D.rps;
    st.m_d = 0;
    st.jptr.assign(st.m_c + 1, 0);
    st.jcol.clear();
    const int iu = N, iL = 2 * N + 1, iV = 2 * N + 2, iS = 2 * N + 3;
    auto x = [&](int i) { return i - 1; };
    auto y = [&](int i) { return N + i; };
    for (int k = 0; k < D.H; ++k) {
        const int b = k * D.ns;
        for (int i = 1; i <= N; ++i) {
            const int row = k * D.rps + i - 1;
            if (k > 0) st.jcol.push_back((k - 1) * D.ns + x(i));
            std::vector<int> cols;
            if (i == 1) cols = {x(1), y(2), iV};
            else if (i < D.Nf) cols = {x(i - 1), x(i), y(i), y(i + 1), iL, iV};
            else if (i == D.Nf) cols = {x(i - 1), x(i), y(i), y(i + 1), iL, iV, iS};
            else if (i < N) cols = {x(i - 1), x(i), y(i), y(i + 1), iV, iS};
            else cols = {x(N - 1), x(N), y(N), iV, iS};
            for (int c : cols) st.jcol.push_back(b + c);
            st.jptr[row + 1] = (int)st.jcol.size();
            if (st.jptr[row + 1] - st.jptr[row] != rx_tray_nnz(D, k, i)) {
                err = "internal: reflux row layout mismatch";
                return false;
            }
        }
        for (int i = 1; i <= N; ++i) {
            const int row = k * D.rps + N + i - 1;
            st.jcol.push_back(b + x(i));
            st.jcol.push_back(b + y(i));
            st.jptr[row + 1] = (int)st.jcol.size();
        }
        const int flow[3][2] = {{iu, iL}, {iL, iV}, {iL, iS}};
        for (int r = 0; r < 3; ++r) {
            st.jcol.push_back(b + flow[r][0]);
            st.jcol.push_back(b + flow[r][1]);
            st.jptr[k * D.rps + 2 * N + r + 1] = (int)st.jcol.size();
        }
    }
    st.jrow.resize(st.jcol.size());
    for (int r = 0; r < st.m_c; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p) st.jrow[p] = r;
    const int ws = rx_wstage(D);
    st.wrow.assign((size_t)ws * D.H, 0);
    st.wcol.assign((size_t)ws * D.H, 0);
    for (int k = 0; k < D.H; ++k) {
        const int o = k * ws, b = k * D.ns;
        auto put = [&](int slot, int r, int c) {
            st.wrow[o + slot] = b + r;
            st.wcol[o + slot] = b + c;
        };
        for (int i = 1; i <= N; ++i) put(i - 1, x(i), x(i));
        put(N, iu, iu);
        for (int j = 1; j < D.Nf; ++j) put(N + j, iL, x(j));
        for (int j = D.Nf; j < N; ++j) put(N + j, iS, x(j));
        put(2 * N, iV, x(1));
        for (int j = 2; j <= N; ++j) put(2 * N + j - 1, iV, y(j));
    }
    st.lb.assign(st.n, 0.0);
    st.ub.assign(st.n, 0.0);
    for (int k = 0; k < D.H; ++k)
        for (int j = 0; j < D.ns; ++j) {
            const int v = k * D.ns + j;
            if (j == iu) {
                st.lb[v] = s.u_lo;
                st.ub[v] = s.u_hi;
            } else if (j >= iL) {
                st.lb[v] = 0.0;
                st.ub[v] = s.flow_hi;
            } else {
                st.lb[v] = s.x_lo;
                st.ub[v] = s.x_hi;
            }
        }
    return true;
}

// Stage-pattern model (eq. 3): the per-stage patterns of the descriptor
// repeated over the horizon.  A state row of stage k > 1 starts with its
// previous-stage columns (lower indices), then its own columns.
static bool build_stage_model(const nmpc_structure& s, Structure& st, std::string& err) {
    const nmpc_stage_model* g = s.stage_model;
    auto bad = [&](const char* what) {
        err = std::string("stage model: ") + what;
        return false;
    };
    if (!g) return bad("NULL descriptor");
    if (s.horizon < 1 || !(s.dt > 0) || !std::isfinite(s.dt) || s.control_horizon != 0)
        return bad("need horizon >= 1, finite dt > 0, control_horizon 0");
    if (g->nx < 1 || g->nu < 1 || g->nu > 16 || g->na < 0 || g->n_alg_rows < 0 || g->n_setpoint < 0 ||
        (g->uses_traj != 0 && g->uses_traj != 1) || g->nw < 0 || g->n_ineq_rows < 0 || g->nw_cross < 0 ||
        g->scratch_per_stage < 0)
        return bad("need nx >= 1, 1 <= nu <= 16, na, n_alg_rows, n_ineq_rows, n_setpoint, nw, nw_cross, "
                   "scratch_per_stage >= 0, uses_traj 0 or 1");
    if (!g->row_ptr || !g->prev_ptr || !g->lb || !g->ub || !g->code_object || g->code_object_size == 0 ||
        g->tag == 0 || (g->nw > 0 && (!g->w_rows || !g->w_cols)) || (g->n_ineq_rows > 0 && !g->ineq_ptr) ||
        (g->nw_cross > 0 && (!g->wx_rows || !g->wx_cols)))
        return bad("missing pattern, bounds, code object or tag");
    const int64_t ns64 = (int64_t)g->nx + g->nu + g->na, rps64 = (int64_t)g->nx + g->n_alg_rows;
    if (ns64 * s.horizon > (int64_t)1 << 30 || (rps64 + g->n_ineq_rows) * s.horizon > (int64_t)1 << 29 ||
        g->nw > (1 << 24) || g->nw_cross > (1 << 24) || g->scratch_per_stage * s.horizon > ((int64_t)1 << 31))
        return bad("problem too large");
    const int ns = (int)ns64, rps = (int)rps64, nx = g->nx, H = s.horizon, nd = g->n_ineq_rows;
    if (g->row_ptr[0] != 0 || g->prev_ptr[0] != 0) return bad("row_ptr / prev_ptr must start at 0");
    for (int r = 0; r < rps; ++r) {
        if (g->row_ptr[r + 1] < g->row_ptr[r] || g->row_ptr[r + 1] - g->row_ptr[r] > ns ||
            g->prev_ptr[r + 1] < g->prev_ptr[r] || g->prev_ptr[r + 1] - g->prev_ptr[r] > nx)
            return bad("row_ptr / prev_ptr not monotone or a row too long");
        if (r >= nx && g->prev_ptr[r + 1] != g->prev_ptr[r]) return bad("an algebraic row uses previous states");
        if (g->row_ptr[r + 1] > g->row_ptr[r] && !g->row_cols) return bad("missing row_cols");
        if (g->prev_ptr[r + 1] > g->prev_ptr[r] && (!g->prev_cols || !g->prev_coef)) return bad("missing prev_cols");
        bool own = false;
        for (int q = g->row_ptr[r]; q < g->row_ptr[r + 1]; ++q) {
            const int c = g->row_cols[q];
            if (c < 0 || c >= ns || (q > g->row_ptr[r] && c <= g->row_cols[q - 1]))
                return bad("row_cols out of range or not strictly ascending");
            own = own || c == r;
        }
        if (r < nx && !own) return bad("a state row does not hold its own state");
        for (int q = g->prev_ptr[r]; q < g->prev_ptr[r + 1]; ++q) {
            const int c = g->prev_cols[q];
            if (c < 0 || c >= nx || (q > g->prev_ptr[r] && c <= g->prev_cols[q - 1]))
                return bad("prev_cols out of range or not strictly ascending");
            if (!std::isfinite(g->prev_coef[q]) || g->prev_coef[q] == 0.0) return bad("prev_coef not finite nonzero");
        }
    }
    if (nd > 0) {
        if (g->ineq_ptr[0] != 0) return bad("ineq_ptr must start at 0");
        for (int r = 0; r < nd; ++r) {
            if (g->ineq_ptr[r + 1] < g->ineq_ptr[r] || g->ineq_ptr[r + 1] - g->ineq_ptr[r] > ns)
                return bad("ineq_ptr not monotone or a row too long");
            if (g->ineq_ptr[r + 1] > g->ineq_ptr[r] && !g->ineq_cols) return bad("missing ineq_cols");
            for (int q = g->ineq_ptr[r]; q < g->ineq_ptr[r + 1]; ++q) {
                const int c = g->ineq_cols[q];
                if (c < 0 || c >= ns || (q > g->ineq_ptr[r] && c <= g->ineq_cols[q - 1]))
                    return bad("ineq_cols out of range or not strictly ascending");
            }
        }
    }
    {
        std::vector<int64_t> keys;
        for (int e = 0; e < g->nw; ++e) {
            const int a = g->w_rows[e], b = g->w_cols[e];
            if (b < 0 || a < b || a >= ns) return bad("Hessian entry out of range or not lower");
            keys.push_back((int64_t)a * ns + b);
        }
        std::sort(keys.begin(), keys.end());
        if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return bad("repeated Hessian entry");
        keys.clear();
        for (int e = 0; e < g->nw_cross; ++e) {
            const int a = g->wx_rows[e], b = g->wx_cols[e];
            if (a < 0 || a >= ns || b < 0 || b >= g->nu) return bad("cross-stage Hessian entry out of range");
            keys.push_back((int64_t)a * g->nu + b);
        }
        std::sort(keys.begin(), keys.end());
        if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) return bad("repeated cross-stage entry");
    }
    for (int j = 0; j < ns; ++j)
        if (std::isnan(g->lb[j]) || std::isnan(g->ub[j]) || !(g->lb[j] < g->ub[j]) || g->lb[j] == INFINITY ||
            g->ub[j] == -INFINITY)
            return bad("bounds must satisfy lb < ub");
    auto& M = st.gm;
    M.ns = ns;
    M.rps = rps;
    M.nsp = g->n_setpoint;
    M.nw = g->nw;
    M.nwx = g->nw_cross;
    M.nd = nd;
    M.traj = g->uses_traj != 0;
    M.tag = g->tag;
    const unsigned char* code = static_cast<const unsigned char*>(g->code_object);
    M.code.assign(code, code + g->code_object_size);
    M.scratch = g->scratch_per_stage;
    // the dense coefficient matrix only when it is not minus the identity
    M.pc_minus_identity = true;
    for (int r = 0; r < nx; ++r)
        if (g->prev_ptr[r + 1] - g->prev_ptr[r] != 1 || g->prev_cols[g->prev_ptr[r]] != r ||
            g->prev_coef[g->prev_ptr[r]] != -1.0)
            M.pc_minus_identity = false;
    M.pc.clear();
    if (!M.pc_minus_identity) {
        if ((int64_t)nx * nx > ((int64_t)1 << 26))
            return bad("state rows whose previous-state coefficients are not minus the identity need nx <= 8192");
        M.pc.assign((size_t)nx * nx, 0.0);
        for (int r = 0; r < nx; ++r)
            for (int q = g->prev_ptr[r]; q < g->prev_ptr[r + 1]; ++q)
                M.pc[(size_t)r * nx + g->prev_cols[q]] = g->prev_coef[q];
    }
    st.nx = nx;
    st.nu = g->nu;
    st.H = H;
    st.n = H * ns;
    st.m_c = H * rps;
    st.m_d = H * nd;
    const int m = st.m_c + st.m_d;
    st.jptr.assign(m + 1, 0);
    st.jcol.clear();
    for (int k = 0; k < H; ++k)
        for (int r = 0; r < rps; ++r) {
            if (k > 0)
                for (int q = g->prev_ptr[r]; q < g->prev_ptr[r + 1]; ++q) st.jcol.push_back((k - 1) * ns + g->prev_cols[q]);
            for (int q = g->row_ptr[r]; q < g->row_ptr[r + 1]; ++q) st.jcol.push_back(k * ns + g->row_cols[q]);
            st.jptr[k * rps + r + 1] = (int)st.jcol.size();
        }
    for (int k = 0; k < H; ++k)
        for (int r = 0; r < nd; ++r) {
            for (int q = g->ineq_ptr[r]; q < g->ineq_ptr[r + 1]; ++q) st.jcol.push_back(k * ns + g->ineq_cols[q]);
            st.jptr[st.m_c + k * nd + r + 1] = (int)st.jcol.size();
        }
    st.jrow.resize(st.jcol.size());
    for (int r = 0; r < m; ++r)
        for (int p = st.jptr[r]; p < st.jptr[r + 1]; ++p) st.jrow[p] = r;
    // Hessian slots: stage 1 its own entries; stage k > 1 its own, then those
    // with the previous stage's controls
    const size_t nwo = (size_t)g->nw, nwx = (size_t)g->nw_cross;
    st.wrow.clear();
    st.wcol.clear();
    for (int k = 0; k < H; ++k) {
        for (size_t e = 0; e < nwo; ++e) {
            st.wrow.push_back(k * ns + g->w_rows[e]);
            st.wcol.push_back(k * ns + g->w_cols[e]);
        }
        if (k > 0)
            for (size_t e = 0; e < nwx; ++e) {
                st.wrow.push_back(k * ns + g->wx_rows[e]);
                st.wcol.push_back((k - 1) * ns + nx + g->wx_cols[e]);
            }
    }
    st.lb.resize(st.n);
    st.ub.resize(st.n);
    for (int k = 0; k < H; ++k)
        for (int j = 0; j < ns; ++j) {
            st.lb[(size_t)k * ns + j] = g->lb[j];
            st.ub[(size_t)k * ns + j] = g->ub[j];
        }
    return true;
}

bool build_structure(const nmpc_structure& s, Structure& out, std::string& err) {
    out = Structure();
    out.desc = s;
    if (s.ordering != NMPC_ORDER_NESTED_DISSECTION && s.ordering != NMPC_ORDER_MIN_DEGREE &&
        s.ordering != NMPC_ORDER_FAMILY_DISSECTION) {
        err = "unknown ordering";
        return false;
    }
    bool ok = false;
    if (s.family == NMPC_FAMILY_DISTILLATION) {
        ok = build_distillation(s, out, err);
    } else if (s.family == NMPC_FAMILY_HEATED_PLATE) {
        ok = build_plate(s, out, err);
    } else if (s.family == NMPC_FAMILY_REFLUX_COLUMN) {
        ok = build_reflux(s, out, err);
    } else if (s.family == NMPC_FAMILY_STAGE_MODEL) {
        ok = build_stage_model(s, out, err);
    } else {
        err = "unsupported problem family";
        return false;
    }
    out.desc.stage_model = nullptr;   // the caller's descriptor is not kept
    if (ok) finish_k_count(out);
    return ok;
}

}  // namespace nmpc
