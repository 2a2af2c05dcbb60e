// SIMD model evaluation (eq. 3): every (stage, variable) pair of the
// distillation transcription is one lane; the stage-major layout makes the
// loads of neighbouring trays and of the previous stage coalesced.  Blocks map
// to instances through the kSpN space, so one launch evaluates a whole batch.
#include "kernels.h"

namespace nmpc {

namespace {

struct Vle {
    double y, yp, ypp;
};

__device__ inline Vle vle(double a, double x) {
    const double g = 1.0 + (a - 1.0) * x;
    Vle v;
    v.y = a * x / g;
    v.yp = a / (g * g);
    v.ypp = -2.0 * a * (a - 1.0) / (g * g * g);
    return v;
}

template <bool Full>
__global__ void __launch_bounds__(kBlock)
k_eval_distill(const InstPtrs* __restrict__ Ia, Space sp, int src, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (I.family != NMPC_FAMILY_DISTILLATION || !ctl_active(I.ctl, pred)) return;
    const DistillDims D = I.dd;
    const DistillConst C = I.dc;
    const int t = lb * kBlock + threadIdx.x;
    if (t >= D.H * D.ns) return;
    const double* __restrict__ y = src == kSrcIter ? I.y : I.yt;
    const double* __restrict__ om = src == kSrcUser ? I.dom : I.om;
    const double* __restrict__ x0 = I.x0;
    const double xD = I.setp[0], xB = I.setp[1];
    double* __restrict__ c = I.c;
    double* __restrict__ d = I.d;
    double* __restrict__ jv = I.jv;
    double* __restrict__ wv = I.wv;
    double* __restrict__ grad = I.grad;
    double* __restrict__ fterm = I.fterm;
    const int32_t* __restrict__ jptr = I.jptr;
    const int mc = I.mc;
    const int k = t / D.ns;
    const int j = t - k * D.ns;
    const double* Y = y + (int64_t)k * D.ns;
    const double R = Y[D.nx], V = Y[D.nx + 1];
    const double dt = C.dt, a = C.alpha, F = C.F;
    if (j < D.nx) {
        const int i = j, N = D.N, fd = D.fd;
        const double xi = Y[i];
        const double xm = i > 0 ? Y[i - 1] : 0.0;
        const double xq = i < D.nx - 1 ? Y[i + 1] : 0.0;
        const double xprev = k > 0 ? y[(int64_t)(k - 1) * D.ns + i] : x0[i];
        const Vle vi = vle(a, xi);
        const Vle vq = vle(a, xq);
        double f, dm = 0.0, dself, dq = 0.0, dR = 0.0, dV;
        if (i == 0) {                       // condenser
            f = V * (vq.y - xi);
            dself = -V;
            dq = V * vq.yp;
            dV = vq.y - xi;
        } else if (i <= N) {                // tray i
            const double lin = i <= fd ? R : R + F;
            const double lout = i < fd ? R : R + F;
            f = lin * xm - lout * xi + V * (vq.y - vi.y);
            if (i == fd) f += F * I.zF[k];
            dm = lin;
            dself = -lout - V * vi.yp;
            dq = V * vq.yp;
            dR = xm - xi;
            dV = vq.y - vi.y;
        } else {                            // reboiler
            f = (R + F) * xm - V * vi.y - (R + F - V) * xi;
            dm = R + F;
            dself = -V * vi.yp - (R + F - V);
            dR = xm - xi;
            dV = -vi.y + xi;
        }
        const int row = k * D.nx + i;
        c[row] = xi - xprev - dt * f;
        double ft = 0.0;
        if (i == 0) ft = (xi - xD) * (xi - xD);
        if (i == D.nx - 1) ft = (xi - xB) * (xi - xB);
        fterm[t] = ft;
        if (Full) {
            int p = jptr[row];
            if (k > 0) jv[p++] = -1.0;
            if (i > 0) jv[p++] = -dt * dm;
            jv[p++] = 1.0 - dt * dself;
            if (i < D.nx - 1) jv[p++] = -dt * dq;
            if (i > 0) jv[p++] = -dt * dR;
            jv[p] = -dt * dV;
            // Hessian slots owned by x_i: sum over the rows that use x_i nonlinearly.
            // Equality multiplier of row (k, r) is omega+ - omega-.
            const double* op = om + (int64_t)k * D.nx;
            const double* on = om + mc + (int64_t)k * D.nx;
            const double li = op[i] - on[i];
            const double lm = i > 0 ? op[i - 1] - on[i - 1] : 0.0;
            const double lq = i < D.nx - 1 ? op[i + 1] - on[i + 1] : 0.0;
            double wdiag = i >= 1 ? -dt * V * vi.ypp * (lm - li) : 0.0;
            if (i == 0 || i == D.nx - 1) wdiag += 2.0;
            const double wR = -dt * ((i <= D.nx - 2 ? lq : 0.0) - (i >= 1 ? li : 0.0));
            double wV;
            if (i == 0) wV = dt * li;
            else if (i <= N) wV = -dt * vi.yp * (lm - li);
            else wV = -dt * (lm * vi.yp + li * (1.0 - vi.yp));
            const int o = k * dl_wstage(D);
            wv[o + i] = wdiag;
            wv[o + D.nx + i] = wR;
            wv[o + 2 * D.nx + 1 + i] = wV;
            grad[t] = i == 0 ? 2.0 * (xi - xD) : (i == D.nx - 1 ? 2.0 * (xi - xB) : 0.0);
        }
    } else {
        const bool isR = j == D.nx;
        const double u = isR ? R : V;
        const double up = k > 0 ? y[(int64_t)(k - 1) * D.ns + j] : I.uprev[j - D.nx];
        const double mv = u - up;
        fterm[t] = C.rho * mv * mv;
        if (isR) d[2 * k] = R - V;
        else d[2 * k + 1] = V - R - F;
        if (k >= D.hc) {   // control horizon: hold u_k = u_{k-1}
            const int row = D.H * D.nx + 2 * (k - D.hc) + (isR ? 0 : 1);
            c[row] = mv;
            if (Full) {
                const int p = jptr[row];
                jv[p] = -1.0;
                jv[p + 1] = 1.0;
            }
        }
        if (Full) {
            const double un = k < D.H - 1 ? y[(int64_t)(k + 1) * D.ns + j] : 0.0;
            grad[t] = 2.0 * C.rho * mv - (k < D.H - 1 ? 2.0 * C.rho * (un - u) : 0.0);
            const int o = k * dl_wstage(D);
            wv[o + (isR ? 2 * D.nx : 3 * D.nx + 1)] = (k == D.H - 1) ? 2.0 * C.rho : 4.0 * C.rho;
            if (k > 0) wv[dl_wcross(D, k) + (isR ? 0 : 1)] = -2.0 * C.rho;
            const int p = jptr[mc + 2 * k + (isR ? 0 : 1)];
            jv[p] = isR ? 1.0 : -1.0;
            jv[p + 1] = isR ? -1.0 : 1.0;
        }
    }
}

// Heated plate: one lane per variable.  A temperature lane evaluates its
// node's residual row, Jacobian row, objective term, gradient and Hessian
// diagonal; a control lane its Hessian diagonal (sum over the nodes its ghost
// cells border).  The flux from q into p is [(T_q - T_p) + kap (T_q^2 - T_p^2)] / h^2.
template <bool Full>
__global__ void __launch_bounds__(kBlock)
k_eval_plate(const InstPtrs* __restrict__ Ia, Space sp, int src, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (I.family != NMPC_FAMILY_HEATED_PLATE || !ctl_active(I.ctl, pred)) return;
    const PlateDims D = I.pd;
    const PlateConst C = I.pc;
    const int t = lb * kBlock + threadIdx.x;
    if (t >= D.H * D.ns) return;
    const double* __restrict__ y = src == kSrcIter ? I.y : I.yt;
    const double* __restrict__ om = src == kSrcUser ? I.dom : I.om;
    const int k = t / D.ns;
    const int l = t - k * D.ns;
    const double* Y = y + (int64_t)k * D.ns;
    const double* U = Y + D.nx;
    const double s2 = C.dt * C.inv_h2;   // dt / h^2
    const double kap = C.kap;
    const int G = D.G, mc = I.mc;
    if (l < D.nx) {
        const int p = l, b = p / G, a = p - b * G;
        const double Tp = Y[p];
        const double Tprev = k > 0 ? y[(int64_t)(k - 1) * D.ns + p] : I.x0[p];
        // neighbours in the Jacobian's column order: interior then ghost (segment order)
        double nbv[4];
        int nn = 0;
        if (b > 0) nbv[nn++] = Y[p - G];
        if (a > 0) nbv[nn++] = Y[p - 1];
        const int n_lo = nn;
        if (a < G - 1) nbv[nn++] = Y[p + 1];
        if (b < G - 1) nbv[nn++] = Y[p + G];
        int sg[2];
        int ng = 0;
        if (b == 0) sg[ng++] = a / D.q;
        if (a == G - 1) sg[ng++] = 4 + b / D.q;
        if (b == G - 1) sg[ng++] = 8 + a / D.q;
        if (a == 0) sg[ng++] = 12 + b / D.q;
        double flux = 0.0;
        for (int e = 0; e < nn; ++e) flux += (nbv[e] - Tp) + kap * (nbv[e] * nbv[e] - Tp * Tp);
        for (int e = 0; e < ng; ++e) {
            const double us = U[sg[e]];
            flux += (us - Tp) + kap * (us * us - Tp * Tp);
        }
        const int row = k * D.nx + p;
        I.c[row] = Tp - Tprev - s2 * flux;
        const double tgt = I.setp[p];
        I.fterm[t] = (Tp - tgt) * (Tp - tgt);
        if (Full) {
            I.grad[t] = 2.0 * (Tp - tgt);
            double* jv = I.jv + I.jptr[row];
            int q = 0;
            if (k > 0) jv[q++] = -1.0;
            for (int e = 0; e < n_lo; ++e) jv[q++] = -s2 * (1.0 + 2.0 * kap * nbv[e]);
            jv[q++] = 1.0 + s2 * (nn + ng) * (1.0 + 2.0 * kap * Tp);
            for (int e = n_lo; e < nn; ++e) jv[q++] = -s2 * (1.0 + 2.0 * kap * nbv[e]);
            for (int e = 0; e < ng; ++e) jv[q++] = -s2 * (1.0 + 2.0 * kap * U[sg[e]]);
            // Hessian diagonal: objective, own row (-kap T_p^2 once per neighbour),
            // interior neighbours' rows (+kap T_p^2 each)
            const double* lp = om + (int64_t)k * D.nx;
            const double* ln = om + mc + (int64_t)k * D.nx;
            double wd = 2.0 + 2.0 * kap * s2 * (nn + ng) * (lp[p] - ln[p]);
            if (b > 0) wd -= 2.0 * kap * s2 * (lp[p - G] - ln[p - G]);
            if (a > 0) wd -= 2.0 * kap * s2 * (lp[p - 1] - ln[p - 1]);
            if (a < G - 1) wd -= 2.0 * kap * s2 * (lp[p + 1] - ln[p + 1]);
            if (b < G - 1) wd -= 2.0 * kap * s2 * (lp[p + G] - ln[p + G]);
            I.wv[t] = wd;
        }
    } else {
        I.fterm[t] = 0.0;
        if (Full) {
            I.grad[t] = 0.0;
            // nodes bordering the ghost cells of segment s
            const int s = l - D.nx, e = s >> 2, j0 = (s & 3) * D.q;
            const double* lp = om + (int64_t)k * D.nx;
            const double* ln = om + mc + (int64_t)k * D.nx;
            double acc = 0.0;
            for (int j = j0; j < j0 + D.q; ++j) {
                const int p = e == 0 ? j : (e == 1 ? j * G + (G - 1) : (e == 2 ? (G - 1) * G + j : j * G));
                acc += lp[p] - ln[p];
            }
            I.wv[t] = -2.0 * kap * s2 * acc;
        }
    }
}

// Reflux column of the case study: one lane per variable of a stage.  A tray
// lane (x_i) evaluates tray i's implicit-Euler row and equilibrium row, their
// Jacobian rows, and the Hessian slots (x_i, x_i), (L, x_i) or (S, x_i) and, for
// tray 1, (V, x_1); a y_i lane the slot (V, y_i); the u, L and V lanes one flow
// row each (L - u D, V - L - D, S - L - F).  Tray rows are c = x_i - x_{i,prev}
// - dt f_i with f the balances of the case study (condenser, rectifying trays,
// feed tray, stripping trays, reboiler); a second derivative of row i's c is
// -dt lam_i times that of f_i, w(i) = -dt lam_i / A_i below.
template <bool Full>
__global__ void __launch_bounds__(kBlock)
k_eval_reflux(const InstPtrs* __restrict__ Ia, Space sp, int src, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (I.family != NMPC_FAMILY_REFLUX_COLUMN || !ctl_active(I.ctl, pred)) return;
    const RefluxDims D = I.rd;
    const RefluxConst C = I.rc;
    const int t = lb * kBlock + threadIdx.x;
    if (t >= D.H * D.ns) return;
    const double* __restrict__ y = src == kSrcIter ? I.y : I.yt;
    const double* __restrict__ om = src == kSrcUser ? I.dom : I.om;
    const int N = D.N, Nf = D.Nf, mc = I.mc;
    const int k = t / D.ns, j = t - k * D.ns;
    const double* Y = y + (int64_t)k * D.ns;
    const double u = Y[N], L = Y[2 * N + 1], V = Y[2 * N + 2], S = Y[2 * N + 3];
    auto X = [&](int i) { return Y[i - 1]; };          // tray i, 1-based
    auto Yv = [&](int i) { return Y[N + i]; };
    const int row0 = k * D.rps;
    // equality multiplier of tray row i of this stage
    auto lam = [&](int i) { return om[row0 + i - 1] - om[mc + row0 + i - 1]; };
    auto hold = [&](int i) { return i == 1 ? C.Ac : (i == N ? C.Ar : C.At); };
    auto w = [&](int i) { return -C.dt * lam(i) / hold(i); };
    double* wv = I.wv + (int64_t)k * rx_wstage(D);
    double ft = 0.0, g = 0.0;
    if (j < N) {
        const int i = j + 1;
        const double xi = X(i);
        const double xprev = k > 0 ? y[(int64_t)(k - 1) * D.ns + j] : I.x0[j];
        // balance f_i and its partials in the row's column order (after x_prev)
        double f, pv[7];
        int np = 0;
        if (i == 1) {
            f = V * (Yv(2) - xi) / C.Ac;
            pv[np++] = -V / C.Ac;                         // x_1
            pv[np++] = V / C.Ac;                          // y_2
            pv[np++] = (Yv(2) - xi) / C.Ac;               // V
        } else if (i < N) {
            const double xm = X(i - 1), yi = Yv(i), yq = Yv(i + 1);
            const double lin = i <= Nf ? L : S;           // liquid from above
            const double lout = i < Nf ? L : S;           // liquid leaving
            f = (lin * xm - lout * xi - V * (yi - yq) + (i == Nf ? C.F * C.xf : 0.0)) / C.At;
            pv[np++] = lin / C.At;                        // x_{i-1}
            pv[np++] = -lout / C.At;                      // x_i
            pv[np++] = -V / C.At;                         // y_i
            pv[np++] = V / C.At;                          // y_{i+1}
            if (i < Nf) {
                pv[np++] = (xm - xi) / C.At;              // L
                pv[np++] = -(yi - yq) / C.At;             // V
            } else if (i == Nf) {
                pv[np++] = xm / C.At;                     // L
                pv[np++] = -(yi - yq) / C.At;             // V
                pv[np++] = -xi / C.At;                    // S
            } else {
                pv[np++] = -(yi - yq) / C.At;             // V
                pv[np++] = (xm - xi) / C.At;              // S
            }
        } else {
            const double xm = X(N - 1), yN = Yv(N);
            f = (S * xm - (C.F - C.D) * xi - V * yN) / C.Ar;
            pv[np++] = S / C.Ar;                          // x_{N-1}
            pv[np++] = -(C.F - C.D) / C.Ar;               // x_N
            pv[np++] = -V / C.Ar;                         // y_N
            pv[np++] = -yN / C.Ar;                        // V
            pv[np++] = xm / C.Ar;                         // S
        }
        const int row = row0 + j;
        I.c[row] = xi - xprev - C.dt * f;
        const double a = C.alpha, gg = 1.0 + (a - 1.0) * xi;
        const int rv = row0 + N + j;
        I.c[rv] = Yv(i) - a * xi / gg;
        if (i == 1) {
            ft = C.dt * (xi - I.setp[0]) * (xi - I.setp[0]);
            g = 2.0 * C.dt * (xi - I.setp[0]);
        }
        if (Full) {
            double* jr = I.jv + I.jptr[row];
            int q = 0;
            if (k > 0) jr[q++] = -1.0;
            const int own = i == 1 ? 0 : 1;              // position of x_i among the partials
            for (int e = 0; e < np; ++e) jr[q++] = -C.dt * pv[e] + (e == own ? 1.0 : 0.0);
            double* je = I.jv + I.jptr[rv];
            je[0] = -a / (gg * gg);
            je[1] = 1.0;
            // Hessian: equilibrium curvature (and the objective on tray 1)
            const double lv = om[rv] - om[mc + rv];
            wv[j] = lv * 2.0 * a * (a - 1.0) / (gg * gg * gg) + (i == 1 ? 2.0 * C.dt : 0.0);
            if (i < Nf) {            // (L, x_i): +w(i+1) from tray i+1, -w(i) from tray i (2 <= i)
                wv[N + i] = w(i + 1) - (i >= 2 ? w(i) : 0.0);
            } else if (i < N) {      // (S, x_i): -w(i) from tray i, +w(i+1) from tray i+1
                wv[N + i] = -w(i) + w(i + 1);
            }
            if (i == 1) wv[2 * N] = -w(1);   // (V, x_1)
        }
    } else if (j == N) {
        I.c[row0 + 2 * N] = L - u * C.D;
        ft = C.dt * C.wu * (u - I.setp[1]) * (u - I.setp[1]);
        g = 2.0 * C.dt * C.wu * (u - I.setp[1]);
        if (Full) {
            double* jr = I.jv + I.jptr[row0 + 2 * N];
            jr[0] = -C.D;
            jr[1] = 1.0;
            wv[N] = 2.0 * C.dt * C.wu;
        }
    } else if (j <= 2 * N) {
        const int i = j - N;
        if (Full && i >= 2) {        // (V, y_i): +w(i-1) from tray i-1, -w(i) from tray i
            wv[2 * N + i - 1] = w(i - 1) - w(i);
        }
    } else if (j == 2 * N + 1) {
        I.c[row0 + 2 * N + 1] = V - L - C.D;
        if (Full) {
            double* jr = I.jv + I.jptr[row0 + 2 * N + 1];
            jr[0] = -1.0;
            jr[1] = 1.0;
        }
    } else if (j == 2 * N + 2) {
        I.c[row0 + 2 * N + 2] = S - L - C.F;
        if (Full) {
            double* jr = I.jv + I.jptr[row0 + 2 * N + 2];
            jr[0] = -1.0;
            jr[1] = 1.0;
        }
    }
    I.fterm[t] = ft;
    if (Full) I.grad[t] = g;
}

}  // namespace

void launch_eval_reflux(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st) {
    if (sp.blocks <= 0) return;
    if (full)
        hipLaunchKernelGGL(k_eval_reflux<true>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
    else
        hipLaunchKernelGGL(k_eval_reflux<false>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
}

void launch_eval_plate(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st) {
    if (sp.blocks <= 0) return;
    if (full)
        hipLaunchKernelGGL(k_eval_plate<true>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
    else
        hipLaunchKernelGGL(k_eval_plate<false>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
}

void launch_eval_distill(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st) {
    if (sp.blocks <= 0) return;
    if (full)
        hipLaunchKernelGGL(k_eval_distill<true>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
    else
        hipLaunchKernelGGL(k_eval_distill<false>, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, src, pred);
}

}  // namespace nmpc
