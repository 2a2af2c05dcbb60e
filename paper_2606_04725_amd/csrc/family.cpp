// Direct transcription of the supported OCP families into fixed sparsity
// patterns (Section 3.1, eqs. 5-6).  Only structure is built here; numeric
// values come from the device eval kernels.
#include <algorithm>
#include <cmath>

#include "distill_layout.h"
#include "plate_layout.h"
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

bool build_structure(const nmpc_structure& s, Structure& out, std::string& err) {
    out = Structure();
    out.desc = s;
    if (s.ordering != NMPC_ORDER_NESTED_DISSECTION && s.ordering != NMPC_ORDER_MIN_DEGREE) {
        err = "unknown ordering";
        return false;
    }
    bool ok = false;
    if (s.family == NMPC_FAMILY_DISTILLATION) {
        ok = build_distillation(s, out, err);
    } else if (s.family == NMPC_FAMILY_HEATED_PLATE) {
        ok = build_plate(s, out, err);
    } else {
        err = "unsupported problem family";
        return false;
    }
    if (ok) finish_k_count(out);
    return ok;
}

}  // namespace nmpc
