// SIMD model evaluation (eq. 3): every (stage, variable) pair of the
// distillation transcription is one lane; the stage-major layout makes the
// loads of neighbouring trays and of the previous stage coalesced.
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
k_eval_distill(DistillDims D, DistillConst C, const double* __restrict__ y, const double* __restrict__ x0,
               const double* __restrict__ zF, const double* __restrict__ uprev, const double* __restrict__ om,
               const int32_t* __restrict__ jptr, int mc, double* __restrict__ c, double* __restrict__ d,
               double* __restrict__ jv, double* __restrict__ wv, double* __restrict__ grad,
               double* __restrict__ fterm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= D.H * D.ns) return;
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
            if (i == fd) f += F * zF[k];
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
        if (i == 0) ft = (xi - C.xD) * (xi - C.xD);
        if (i == D.nx - 1) ft = (xi - C.xB) * (xi - C.xB);
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
            grad[t] = i == 0 ? 2.0 * (xi - C.xD) : (i == D.nx - 1 ? 2.0 * (xi - C.xB) : 0.0);
        }
    } else {
        const bool isR = j == D.nx;
        const double u = isR ? R : V;
        const double up = k > 0 ? y[(int64_t)(k - 1) * D.ns + j] : uprev[j - D.nx];
        const double mv = u - up;
        fterm[t] = C.rho * mv * mv;
        if (isR) d[2 * k] = R - V;
        else d[2 * k + 1] = V - R - F;
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

}  // namespace

void launch_eval_distill(bool full, const DistillDims& D, const DistillConst& C, const double* y,
                         const double* x0, const double* zF, const double* uprev, const double* om,
                         const int32_t* jptr, int mc, double* c, double* d, double* jv, double* wv,
                         double* grad, double* fterm, hipStream_t st) {
    const int total = D.H * D.ns;
    const int blocks = (total + kBlock - 1) / kBlock;
    if (full)
        hipLaunchKernelGGL(k_eval_distill<true>, dim3(blocks), dim3(kBlock), 0, st, D, C, y, x0, zF, uprev, om,
                           jptr, mc, c, d, jv, wv, grad, fterm);
    else
        hipLaunchKernelGGL(k_eval_distill<false>, dim3(blocks), dim3(kBlock), 0, st, D, C, y, x0, zF, uprev,
                           om, jptr, mc, c, d, jv, wv, grad, fterm);
}

}  // namespace nmpc
