// Device buffers, IPM vector kernels and the host-side driver of Algorithm 2.
//
// Every step of an iteration runs on the GPU: model evaluation, residuals and
// optimality errors (eqs. 11, 27-28), condensed assembly (eqs. 14, 17), the
// supernodal factorization with inertia correction (eqs. 12-13, 20-21), the
// forward/back solves (eqs. 22-25), recovery of the other directions, the
// fraction-to-boundary rule and the line search (eq. 26).  The host reads a
// handful of reduced scalars per phase to take the same decisions as the
// method's description: barrier update, regularization, step acceptance.
//
// Reductions are two-level and deterministic: each block reduces its slice in
// a fixed tree order into a partial buffer, then one block reduces the
// partials in block order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace nmpc {

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return NMPC_ERR_HIP;                                                      \
        }                                                                             \
    } while (0)

namespace {

constexpr int kMaxQ = 12;
enum Op : int { kSum = 0, kMax = 1, kMin = 2 };

__device__ inline double combine(int op, double a, double b) {
    return op == kSum ? a + b : (op == kMax ? fmax(a, b) : fmin(a, b));
}

struct Ops {
    int q;
    int op[kMaxQ];
};

constexpr int kWaves = kBlock / 64;

// Butterfly reduction across the 64 lanes of a wave (fixed pattern).
__device__ inline double wave_reduce(double v, int op) {
    for (int off = 32; off > 0; off >>= 1) v = combine(op, v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce every quantity over the block (waves, then the per-wave results in
// wave order) and let thread q write quantity q's block result to part.
__device__ void store_partials(const double* v, const Ops& ops, double* part, int nblk, double* sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < ops.q; ++q) {
        const double r = wave_reduce(v[q], ops.op[q]);
        if (lane == 0) sh[q * kWaves + wv] = r;
    }
    __syncthreads();
    if ((int)threadIdx.x < ops.q) {
        const int q = threadIdx.x;
        double acc = sh[q * kWaves];
        for (int w = 1; w < kWaves; ++w) acc = combine(ops.op[q], acc, sh[q * kWaves + w]);
        part[(int64_t)q * nblk + blockIdx.x] = acc;
    }
}

__device__ inline double ident(int op) {
    return op == kSum ? 0.0 : (op == kMax ? -INFINITY : INFINITY);
}

__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ part, int nblk, Ops ops,
                                                      double* __restrict__ out) {
    __shared__ double sh[kMaxQ * kWaves];
    double v[kMaxQ];
    for (int q = 0; q < ops.q; ++q) {
        double acc = ident(ops.op[q]);
        for (int b = threadIdx.x; b < nblk; b += kBlock) acc = combine(ops.op[q], acc, part[(int64_t)q * nblk + b]);
        v[q] = acc;
    }
    store_partials(v, ops, out, 1, sh);
}

struct Vec {
    int n, mc, md, ml;
    double gamma;
    const double* lb;
    const double* ub;
};

__device__ inline bool hasL(const Vec& V, int j) { return V.lb[j] > -INFINITY; }
__device__ inline bool hasU(const Vec& V, int j) { return V.ub[j] < INFINITY; }

__device__ inline double lifted_g(const Vec& V, const double* c, const double* d, int r) {
    if (r < V.mc) return c[r] - V.gamma;
    if (r < 2 * V.mc) return -c[r - V.mc] - V.gamma;
    return d[r - 2 * V.mc];
}

// ---- phase A: optimality-error ingredients at the current iterate --------------
// q: 0 f(sum) 1 dual(max) 2 |omega-beta|(max) 3 |g+s|(max) 4 sb max 5 sb min
//    6 gL zL max 7 gL zL min 8 gU zU max 9 gU zU min 10 non-finite count(sum)
__global__ void __launch_bounds__(kBlock)
k_phaseA(Vec V, const double* __restrict__ y, const double* __restrict__ s, const double* __restrict__ om,
         const double* __restrict__ be, const double* __restrict__ zl, const double* __restrict__ zu,
         const double* __restrict__ grad, const double* __restrict__ fterm, const double* __restrict__ c,
         const double* __restrict__ d, const double* __restrict__ jv, const int32_t* __restrict__ jt_ptr,
         const int32_t* __restrict__ jt_slot, const int32_t* __restrict__ jt_row, double* __restrict__ gtw,
         double* __restrict__ part, Ops ops) {
    __shared__ double sh[kMaxQ * kWaves];
    double q[11] = {0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, 0.0};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < V.n) {
        const int j = t;
        double acc = 0.0;
        for (int e = jt_ptr[j]; e < jt_ptr[j + 1]; ++e) {
            const int r = jt_row[e];
            const double lam = r < V.mc ? om[r] - om[V.mc + r] : om[V.mc + r];
            acc += jv[jt_slot[e]] * lam;
        }
        gtw[j] = acc;
        const bool hl = hasL(V, j), hu = hasU(V, j);
        const double dual = grad[j] + acc - (hl ? zl[j] : 0.0) + (hu ? zu[j] : 0.0);
        q[0] = fterm[j];
        q[1] = fabs(dual);
        if (hl) {
            const double p = (y[j] - V.lb[j]) * zl[j];
            q[6] = p;
            q[7] = p;
        }
        if (hu) {
            const double p = (V.ub[j] - y[j]) * zu[j];
            q[8] = p;
            q[9] = p;
        }
        if (!isfinite(fterm[j]) || !isfinite(grad[j])) q[10] = 1.0;
    } else if (t < V.n + V.ml) {
        const int r = t - V.n;
        const double g = lifted_g(V, c, d, r);
        q[2] = fabs(om[r] - be[r]);
        q[3] = fabs(g + s[r]);
        q[4] = s[r] * be[r];
        q[5] = q[4];
        if (!isfinite(g)) q[10] = 1.0;
    }
    store_partials(q, ops, part, gridDim.x, sh);
}

// ---- phase B: condensed system ingredients --------------------------------------
// per original row r: lifted Q, r2, r4 and their combinations
//   c row r:  qeff = Q+ + Q-,  vcomb = (Q+ r4+ - r2+) - (Q- r4- - r2-)
//   d row r:  qeff = Q,        vcomb = Q r4 - r2
__global__ void __launch_bounds__(kBlock)
k_rows_prep(Vec V, double mu, const double* __restrict__ s, const double* __restrict__ om,
            const double* __restrict__ be, const double* __restrict__ c, const double* __restrict__ d,
            double* __restrict__ Q, double* __restrict__ r2, double* __restrict__ r4, double* __restrict__ qeff,
            double* __restrict__ vcomb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = V.mc + V.md;
    if (r >= m) return;
    if (r < V.mc) {
        const int a = r, b = V.mc + r;
        const double Qa = be[a] / s[a], Qb = be[b] / s[b];
        const double r2a = om[a] - mu / s[a], r2b = om[b] - mu / s[b];
        const double r4a = lifted_g(V, c, d, a) + s[a], r4b = lifted_g(V, c, d, b) + s[b];
        Q[a] = Qa; Q[b] = Qb;
        r2[a] = r2a; r2[b] = r2b;
        r4[a] = r4a; r4[b] = r4b;
        qeff[r] = Qa + Qb;
        vcomb[r] = (Qa * r4a - r2a) - (Qb * r4b - r2b);
    } else {
        const int a = V.mc + r;
        const double Qa = be[a] / s[a];
        const double r2a = om[a] - mu / s[a];
        const double r4a = lifted_g(V, c, d, a) + s[a];
        Q[a] = Qa; r2[a] = r2a; r4[a] = r4a;
        qeff[r] = Qa;
        vcomb[r] = Qa * r4a - r2a;
    }
}

// per variable: Sigma, and rhs = -r1 - G^T (Q r4 - r2), r1 = grad + G^T omega - mu/gL + mu/gU
__global__ void __launch_bounds__(kBlock)
k_var_prep(Vec V, double mu, const double* __restrict__ y, const double* __restrict__ zl,
           const double* __restrict__ zu, const double* __restrict__ grad, const double* __restrict__ gtw,
           const double* __restrict__ jv, const int32_t* __restrict__ jt_ptr, const int32_t* __restrict__ jt_slot,
           const int32_t* __restrict__ jt_row, const double* __restrict__ vcomb, double* __restrict__ sig,
           double* __restrict__ rhs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= V.n) return;
    const bool hl = hasL(V, j), hu = hasU(V, j);
    const double gl = hl ? y[j] - V.lb[j] : 1.0;
    const double gu = hu ? V.ub[j] - y[j] : 1.0;
    sig[j] = (hl ? zl[j] / gl : 0.0) + (hu ? zu[j] / gu : 0.0);
    const double r1 = grad[j] + gtw[j] - (hl ? mu / gl : 0.0) + (hu ? mu / gu : 0.0);
    double acc = 0.0;
    for (int e = jt_ptr[j]; e < jt_ptr[j + 1]; ++e) acc += jv[jt_slot[e]] * vcomb[jt_row[e]];
    rhs[j] = -r1 - acc;
}

// K slot values: W + Sigma + J^T diag(qeff) J, gathered per slot (no atomics)
__global__ void __launch_bounds__(kBlock)
k_assemble(int64_t nk, const int32_t* __restrict__ wslot, const int32_t* __restrict__ kdiag,
           const int32_t* __restrict__ kc_ptr, const int32_t* __restrict__ kc_a, const int32_t* __restrict__ kc_b,
           const int32_t* __restrict__ kc_r, const double* __restrict__ wv, const double* __restrict__ sig,
           const double* __restrict__ jv, const double* __restrict__ qeff, double* __restrict__ kv) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nk) return;
    const int ws = wslot[t], dg = kdiag[t];
    double v = ws >= 0 ? wv[ws] : 0.0;
    if (dg >= 0) v += sig[dg];
    for (int e = kc_ptr[t]; e < kc_ptr[t + 1]; ++e) v += jv[kc_a[e]] * qeff[kc_r[e]] * jv[kc_b[e]];
    kv[t] = v;
}

__device__ inline double ftb(double v, double dv, double tau) { return dv < 0.0 ? (-tau * v) / dv : INFINITY; }

// ---- phase E: remaining directions and step / merit ingredients ------------------
// q: 0 alpha_primal(min) 1 alpha_dual(min) 2 |omega+domega|(max) 3 grad.dy 4 sum ds/s
//    5 sum dy/gL 6 sum dy/gU 7 |r4|_1 8 sum ln s 9 sum ln gL 10 sum ln gU
__global__ void __launch_bounds__(kBlock)
k_phaseE(Vec V, double mu, double tau, const double* __restrict__ y, const double* __restrict__ s,
         const double* __restrict__ om, const double* __restrict__ be, const double* __restrict__ zl,
         const double* __restrict__ zu, const double* __restrict__ grad, const double* __restrict__ dy,
         const double* __restrict__ Q, const double* __restrict__ r2, const double* __restrict__ r4,
         const double* __restrict__ jv, const int32_t* __restrict__ jptr, const int32_t* __restrict__ jcol,
         double* __restrict__ ds, double* __restrict__ dom, double* __restrict__ dbe, double* __restrict__ dzl,
         double* __restrict__ dzu, double* __restrict__ part, Ops ops) {
    __shared__ double sh[kMaxQ * kWaves];
    double q[11] = {INFINITY, INFINITY, -INFINITY, 0, 0, 0, 0, 0, 0, 0, 0};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = V.mc + V.md;
    if (t < m) {
        const int r = t;
        double jdy = 0.0;
        for (int p = jptr[r]; p < jptr[r + 1]; ++p) jdy += jv[p] * dy[jcol[p]];
        const int nl = r < V.mc ? 2 : 1;
        for (int h = 0; h < nl; ++h) {
            const int l = r < V.mc ? (h == 0 ? r : V.mc + r) : V.mc + r;
            const double sgn = (r < V.mc && h == 1) ? -1.0 : 1.0;
            const double dsl = -r4[l] - sgn * jdy;
            const double doml = -r2[l] - Q[l] * dsl;
            const double dbel = mu / s[l] - be[l] - Q[l] * dsl;
            ds[l] = dsl;
            dom[l] = doml;
            dbe[l] = dbel;
            q[0] = fmin(q[0], ftb(s[l], dsl, tau));
            q[1] = fmin(q[1], ftb(be[l], dbel, tau));
            q[2] = fmax(q[2], fabs(om[l] + doml));
            q[4] += dsl / s[l];
            q[7] += fabs(r4[l]);
            q[8] += log(s[l]);
        }
    } else if (t < m + V.n) {
        const int j = t - m;
        const bool hl = hasL(V, j), hu = hasU(V, j);
        const double gl = hl ? y[j] - V.lb[j] : 1.0;
        const double gu = hu ? V.ub[j] - y[j] : 1.0;
        const double dyj = dy[j];
        const double dzlj = hl ? mu / gl - zl[j] - (zl[j] / gl) * dyj : 0.0;
        const double dzuj = hu ? mu / gu - zu[j] + (zu[j] / gu) * dyj : 0.0;
        dzl[j] = dzlj;
        dzu[j] = dzuj;
        q[3] = grad[j] * dyj;
        if (hl) {
            q[0] = fmin(q[0], ftb(gl, dyj, tau));
            q[1] = fmin(q[1], ftb(zl[j], dzlj, tau));
            q[5] = dyj / gl;
            q[9] = log(gl);
        }
        if (hu) {
            q[0] = fmin(q[0], ftb(gu, -dyj, tau));
            q[1] = fmin(q[1], ftb(zu[j], dzuj, tau));
            q[6] = dyj / gu;
            q[10] = log(gu);
        }
    }
    store_partials(q, ops, part, gridDim.x, sh);
}

__global__ void __launch_bounds__(kBlock)
k_trial_point(int n, int ml, double alpha, const double* __restrict__ y, const double* __restrict__ dy,
              const double* __restrict__ s, const double* __restrict__ ds, double* __restrict__ yt,
              double* __restrict__ st) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) yt[t] = y[t] + alpha * dy[t];
    if (t < ml) st[t] = s[t] + alpha * ds[t];
}

// merit ingredients at the trial point
// q: 0 f(sum) 1 sum ln s 2 sum ln gL 3 sum ln gU 4 |g+s|_1 5 non-finite count
__global__ void __launch_bounds__(kBlock)
k_phaseT(Vec V, const double* __restrict__ yt, const double* __restrict__ st, const double* __restrict__ fterm,
         const double* __restrict__ c, const double* __restrict__ d, double* __restrict__ part, Ops ops) {
    __shared__ double sh[kMaxQ * kWaves];
    double q[6] = {0, 0, 0, 0, 0, 0};
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < V.n) {
        const int j = t;
        q[0] = fterm[j];
        if (hasL(V, j)) q[2] = log(yt[j] - V.lb[j]);
        if (hasU(V, j)) q[3] = log(V.ub[j] - yt[j]);
        if (!isfinite(fterm[j])) q[5] = 1.0;
    } else if (t < V.n + V.ml) {
        const int r = t - V.n;
        const double g = lifted_g(V, c, d, r);
        q[1] = log(st[r]);
        q[4] = fabs(g + st[r]);
        if (!isfinite(g)) q[5] = 1.0;
    }
    store_partials(q, ops, part, gridDim.x, sh);
}

// z <- z + alpha dz, then keep beta, zL, zU within kappa_sigma of mu / (slack or gap)
__global__ void __launch_bounds__(kBlock)
k_update(Vec V, double alpha, double mu, double ks, double* __restrict__ y, double* __restrict__ s,
         double* __restrict__ om, double* __restrict__ be, double* __restrict__ zl, double* __restrict__ zu,
         const double* __restrict__ dy, const double* __restrict__ ds, const double* __restrict__ dom,
         const double* __restrict__ dbe, const double* __restrict__ dzl, const double* __restrict__ dzu) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < V.n) {
        const int j = t;
        const double yn = y[j] + alpha * dy[j];
        y[j] = yn;
        if (hasL(V, j)) {
            const double gl = yn - V.lb[j];
            const double z = zl[j] + alpha * dzl[j];
            zl[j] = fmin(fmax(z, mu / (ks * gl)), ks * mu / gl);
        } else {
            zl[j] = 0.0;
        }
        if (hasU(V, j)) {
            const double gu = V.ub[j] - yn;
            const double z = zu[j] + alpha * dzu[j];
            zu[j] = fmin(fmax(z, mu / (ks * gu)), ks * mu / gu);
        } else {
            zu[j] = 0.0;
        }
    }
    if (t < V.ml) {
        const int r = t;
        const double sn = s[r] + alpha * ds[r];
        s[r] = sn;
        om[r] = om[r] + alpha * dom[r];
        const double b = be[r] + alpha * dbe[r];
        be[r] = fmin(fmax(b, mu / (ks * sn)), ks * mu / sn);
    }
}

// cold start: push y into the bounds' interior (bound_push of magnitude and range)
__global__ void __launch_bounds__(kBlock)
k_push_bounds(Vec V, double bp, double* __restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= V.n) return;
    const bool hl = hasL(V, j), hu = hasU(V, j);
    double pl = hl ? bp * fmax(1.0, fabs(V.lb[j])) : 0.0;
    double pu = hu ? bp * fmax(1.0, fabs(V.ub[j])) : 0.0;
    if (hl && hu) {
        const double rng = V.ub[j] - V.lb[j];
        pl = fmin(pl, 0.5 * bp * rng);
        pu = fmin(pu, 0.5 * bp * rng);
    }
    double v = y[j];
    if (hl) v = fmax(v, V.lb[j] + pl);
    if (hu) v = fmin(v, V.ub[j] - pu);
    y[j] = v;
}

// cold start: slacks, multipliers centred at mu0
__global__ void __launch_bounds__(kBlock)
k_cold_duals(Vec V, double mu0, double sp, const double* __restrict__ c, const double* __restrict__ d,
             const double* __restrict__ y, double* __restrict__ s, double* __restrict__ om, double* __restrict__ be,
             double* __restrict__ zl, double* __restrict__ zu) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < V.ml) {
        const double g = lifted_g(V, c, d, t);
        const double sv = fmax(-g, sp * fmax(1.0, fabs(g)));
        s[t] = sv;
        om[t] = 0.0;
        be[t] = mu0 / sv;
    }
    if (t < V.n) {
        zl[t] = hasL(V, t) ? mu0 / (y[t] - V.lb[t]) : 0.0;
        zu[t] = hasU(V, t) ? mu0 / (V.ub[t] - y[t]) : 0.0;
    }
}

__global__ void k_clear_flag(int* __restrict__ flag) { *flag = 0; }

// ---- sensitivities ------------------------------------------------------------------
constexpr int kMaxSeed = 16;
struct Seed {
    double u[kMaxSeed];
};

// rhs = seed_obj * grad f + S_u^T seed_u (first-stage controls at positions iu0 .. iu0 + nu)
__global__ void __launch_bounds__(kBlock)
k_adj_seed(int n, int iu0, int nu, const double* __restrict__ grad, double seed_obj, Seed seed,
           double* __restrict__ rhs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double v = seed_obj * grad[j];
    if (j >= iu0 && j < iu0 + nu) v += seed.u[j - iu0];
    rhs[j] = v;
}

// Parameter contractions of w = K^{-1} seed for the distillation family (one block):
//   x0:       (Q+ + Q-) (J w) on the stage-1 rows
//   zF_k:     dt F (Q+ + Q-) (J w) on the feed-tray row of stage k
//   xD*, xB*: 2 sum_k w(top|bottom state) - 2 seed_obj sum_k (state - setpoint)
//   u_prev:   2 rho w(u_1) - 2 rho seed_obj (u_1 - u_prev)
// out = [x0 (nx) | setpoint (2) | traj (H) | u_prev (2)]
__global__ void __launch_bounds__(kBlock)
k_adj_gather_distill(DistillDims D, DistillConst C, const double* __restrict__ y, const double* __restrict__ uprev,
                     const double* __restrict__ w, const double* __restrict__ jv, const int32_t* __restrict__ jptr,
                     const int32_t* __restrict__ jcol, const double* __restrict__ qeff, double seed_obj,
                     double* __restrict__ out) {
    __shared__ double sh[kMaxQ * kWaves];
    const int tid = threadIdx.x;
    for (int t = tid; t < D.nx + D.H; t += kBlock) {
        const int r = t < D.nx ? t : (t - D.nx) * D.nx + D.fd;
        double jw = 0.0;
        for (int q = jptr[r]; q < jptr[r + 1]; ++q) jw += jv[q] * w[jcol[q]];
        const double v = qeff[r] * jw;
        if (t < D.nx) out[t] = v;
        else out[D.nx + 2 + (t - D.nx)] = C.dt * C.F * v;
    }
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < D.H; k += kBlock) {
        const int top = k * D.ns, bot = k * D.ns + D.nx - 1;
        a[0] += w[top];
        a[1] += y[top] - C.xD;
        a[2] += w[bot];
        a[3] += y[bot] - C.xB;
    }
    Ops ops{4, {kSum, kSum, kSum, kSum}};
    store_partials(a, ops, sh + 4 * kWaves, 1, sh);   // block sums land in sh[4 kWaves .. 4 kWaves + 4)
    __syncthreads();
    if (tid == 0) {
        const double* r = sh + 4 * kWaves;
        out[D.nx] = 2.0 * r[0] - 2.0 * seed_obj * r[1];
        out[D.nx + 1] = 2.0 * r[2] - 2.0 * seed_obj * r[3];
    }
    if (tid < 2) {
        const int iu = D.nx + tid;
        out[D.nx + 2 + D.H + tid] = 2.0 * C.rho * w[iu] - 2.0 * C.rho * seed_obj * (y[iu] - uprev[tid]);
    }
}

inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

// ==================================================================================
struct Device {
    hipStream_t stream = nullptr;
    int n = 0, mc = 0, md = 0, ml = 0, m = 0;
    int64_t nnzj = 0, nnzw = 0, nnzk = 0;
    DistillDims dd{};
    DistillConst dc{};
    Vec vec{};
    // structure
    int32_t *jptr = nullptr, *jcol = nullptr, *jt_ptr = nullptr, *jt_slot = nullptr, *jt_row = nullptr;
    double *lb = nullptr, *ub = nullptr;
    // symbolic
    int32_t *perm = nullptr, *sn_ptr = nullptr, *rows = nullptr, *child_ptr = nullptr, *child_list = nullptr;
    int32_t *level_list = nullptr, *rel = nullptr, *k_ptr = nullptr, *k_fpos = nullptr;
    int64_t *rows_ptr = nullptr, *l_off = nullptr, *u_off = nullptr, *uv_off = nullptr, *rel_off = nullptr;
    int32_t *k_wslot = nullptr, *k_diag = nullptr, *kc_ptr = nullptr, *kc_a = nullptr, *kc_b = nullptr,
            *kc_r = nullptr;
    // launch schedule of the supernodal tree: forward (leaves to root) and backward
    struct Launch {
        int gptr_off, groups;
        size_t lds_factor, lds_solve, lds_vec;
    };
    std::vector<Launch> fwd_launches, bwd_launches;
    int32_t *sched_nodes = nullptr, *sched_gptr = nullptr;
    bool front_in_lds = true;
    double* gscratch = nullptr;
    int64_t gstride = 0;
    SnView S{};
    // parameters
    double *x0 = nullptr, *zF = nullptr, *uprev = nullptr;
    // iterate and work
    double *y = nullptr, *s = nullptr, *om = nullptr, *be = nullptr, *zl = nullptr, *zu = nullptr;
    double *c = nullptr, *d = nullptr, *jv = nullptr, *wv = nullptr, *grad = nullptr, *fterm = nullptr;
    double *gtw = nullptr, *sig = nullptr, *rhs = nullptr, *dy = nullptr, *xp = nullptr;
    double *Q = nullptr, *r2 = nullptr, *r4 = nullptr, *qeff = nullptr, *vcomb = nullptr;
    double *ds = nullptr, *dom = nullptr, *dbe = nullptr, *dzl = nullptr, *dzu = nullptr;
    double *yt = nullptr, *st = nullptr;
    double *kv = nullptr, *L = nullptr, *U = nullptr, *uvec = nullptr;
    int* fail = nullptr;
    double *part = nullptr, *scal = nullptr;
    double* hscal = nullptr;   // pinned
    int* hfail = nullptr;      // pinned
    int part_blocks = 0;
    int max_width = 0;
    std::vector<void*> allocs;
    hipEvent_t ev[10] = {};
    // sensitivities: factor of K at the returned iterate, kept until it changes
    bool adj_ready = false;
    double adj_eta = 0.0;
    double *adj_rhs = nullptr, *adj_w = nullptr, *adj_out = nullptr;   // phase timers: eval, assemble, factor, solve, line search (start, end)
};

namespace {

template <class T>
hipError_t dalloc(Device& D, T*& p, size_t count) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        D.allocs.push_back(v);
        p = static_cast<T*>(v);
    }
    return e;
}

template <class T>
hipError_t upload(Device& D, T*& p, const std::vector<T>& h) {
    hipError_t e = dalloc(D, p, h.size());
    if (e != hipSuccess) return e;
    if (!h.empty()) e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

}  // namespace

bool device_present() {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess) return false;
    return cnt > 0;
}

void device_free(Problem& p) {
    if (!p.dev) return;
    Device& D = *p.dev;
    for (void* a : D.allocs) (void)hipFree(a);
    if (D.hscal) (void)hipHostFree(D.hscal);
    if (D.hfail) (void)hipHostFree(D.hfail);
    for (auto evv : D.ev)
        if (evv) (void)hipEventDestroy(evv);
    if (D.stream) (void)hipStreamDestroy(D.stream);
    delete p.dev;
    p.dev = nullptr;
}

nmpc_status device_init(Problem& p, std::string& err) {
    if (p.dev) return NMPC_OK;
    const Structure& st = p.st;
    const Symbolic& sy = p.sym;
    p.dev = new Device();
    Device& D = *p.dev;
    auto fail_cleanup = [&](nmpc_status rc) {
        device_free(p);
        return rc;
    };
    hipError_t e = hipStreamCreate(&D.stream);
    if (e != hipSuccess) {
        err = std::string("hipStreamCreate: ") + hipGetErrorString(e);
        return fail_cleanup(NMPC_ERR_HIP);
    }
    D.n = st.n;
    D.mc = st.m_c;
    D.md = st.m_d;
    D.ml = 2 * st.m_c + st.m_d;
    D.m = st.m_c + st.m_d;
    D.nnzj = (int64_t)st.jcol.size();
    D.nnzw = (int64_t)st.wrow.size();
    D.nnzk = (int64_t)sy.k_fpos.size();
    const nmpc_structure& s = st.desc;
    D.dd.N = s.n_trays;
    D.dd.nx = s.n_trays + 2;
    D.dd.ns = s.n_trays + 4;
    D.dd.H = s.horizon;
    D.dd.fd = s.n_trays / 2;
    D.dc.dt = s.dt;
    D.dc.alpha = s.alpha;
    D.dc.F = s.feed_flow;
    D.dc.rho = s.move_penalty;
    // LDS budget of the fronts
    int dev = 0, lds_max = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    const size_t lds_limit = (size_t)lds_max;
    // Schedule: every level below the narrow top is one launch with one group per
    // supernode; the top levels that hold at most kTailWidth supernodes each form
    // a single group walked by one workgroup (a chain costs one launch).
    constexpr int kTailWidth = 2;
    int tail = sy.depth;
    while (tail > 0 && sy.level_ptr[tail] - sy.level_ptr[tail - 1] <= kTailWidth) --tail;
    if (sy.depth - tail < 2) tail = sy.depth;
    std::vector<int32_t> nodes, gptr;
    auto sizes = [&](int sn, size_t& fac, size_t& sol, size_t& vec) {
        const size_t mr = (size_t)(sy.sn_rows_ptr[sn + 1] - sy.sn_rows_ptr[sn]);
        const size_t w = (size_t)(sy.sn_ptr[sn + 1] - sy.sn_ptr[sn]);
        fac = std::max(fac, mr * (mr | 1) * sizeof(double) + kRelInts * sizeof(int32_t));
        sol = std::max(sol, (mr * (w | 1) + mr + 2 * w) * sizeof(double));
        vec = std::max(vec, mr * sizeof(double));
    };
    auto add_launch = [&](std::vector<Device::Launch>& out, const std::vector<std::vector<int32_t>>& groups) {
        Device::Launch L{(int)gptr.size(), (int)groups.size(), 0, 0, 0};
        for (const auto& g : groups) {
            gptr.push_back((int32_t)nodes.size());
            for (int32_t sn : g) {
                nodes.push_back(sn);
                sizes(sn, L.lds_factor, L.lds_solve, L.lds_vec);
            }
        }
        gptr.push_back((int32_t)nodes.size());
        out.push_back(L);
    };
    std::vector<int32_t> tail_nodes;
    for (int Lv = tail; Lv < sy.depth; ++Lv)
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) tail_nodes.push_back(sy.level_list[i]);
    for (int Lv = 0; Lv < tail; ++Lv) {
        std::vector<std::vector<int32_t>> g;
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) g.push_back({sy.level_list[i]});
        add_launch(D.fwd_launches, g);
    }
    if (!tail_nodes.empty()) add_launch(D.fwd_launches, {tail_nodes});
    if (!tail_nodes.empty()) add_launch(D.bwd_launches, {std::vector<int32_t>(tail_nodes.rbegin(), tail_nodes.rend())});
    for (int Lv = tail - 1; Lv >= 0; --Lv) {
        std::vector<std::vector<int32_t>> g;
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) g.push_back({sy.level_list[i]});
        add_launch(D.bwd_launches, g);
    }
    size_t need_factor = 0, need_solve = 0;
    for (const auto& L : D.fwd_launches) {
        need_factor = std::max(need_factor, L.lds_factor);
        need_solve = std::max(need_solve, L.lds_solve);
    }
    D.front_in_lds = need_factor <= lds_limit;
    if (sy.max_front > kRelInts) {
        err = "front larger than the relative-position buffer; unsupported front size";
        return fail_cleanup(NMPC_ERR_UNSUPPORTED);
    }
    if (need_solve > lds_limit) {
        err = "supernode panel exceeds shared memory; unsupported front size";
        return fail_cleanup(NMPC_ERR_UNSUPPORTED);
    }
    for (int sn = 0; sn < sy.nsn; ++sn) D.max_width = std::max(D.max_width, sy.sn_ptr[sn + 1] - sy.sn_ptr[sn]);

    int max_groups = 0;
    for (const auto& L : D.fwd_launches) max_groups = std::max(max_groups, L.groups);
    e = linalg_configure(std::min(lds_limit, std::max(need_factor, need_solve)));
    if (e != hipSuccess) {
        err = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
        return fail_cleanup(NMPC_ERR_HIP);
    }
#define UP(ptr, vec)                                                      \
    if ((e = upload(D, ptr, vec)) != hipSuccess) {                        \
        err = std::string("upload " #vec ": ") + hipGetErrorString(e);    \
        return fail_cleanup(e == hipErrorOutOfMemory ? NMPC_ERR_OOM : NMPC_ERR_HIP); \
    }
#define AL(ptr, count)                                                    \
    if ((e = dalloc(D, ptr, count)) != hipSuccess) {                      \
        err = std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e); \
        return fail_cleanup(e == hipErrorOutOfMemory ? NMPC_ERR_OOM : NMPC_ERR_HIP); \
    }
    UP(D.jptr, st.jptr);
    UP(D.jcol, st.jcol);
    UP(D.jt_ptr, sy.jt_ptr);
    UP(D.jt_slot, sy.jt_slot);
    UP(D.jt_row, sy.jt_row);
    std::vector<double> lbv(st.lb), ubv(st.ub);
    UP(D.lb, lbv);
    UP(D.ub, ubv);
    UP(D.perm, sy.perm);
    UP(D.sn_ptr, sy.sn_ptr);
    UP(D.rows_ptr, sy.sn_rows_ptr);
    UP(D.rows, sy.sn_rows);
    UP(D.child_ptr, sy.child_ptr);
    UP(D.child_list, sy.child_list);
    UP(D.sched_nodes, nodes);
    UP(D.sched_gptr, gptr);
    UP(D.l_off, sy.l_off);
    UP(D.u_off, sy.u_off);
    UP(D.uv_off, sy.uv_off);
    UP(D.rel_off, sy.rel_off);
    UP(D.rel, sy.rel);
    UP(D.k_ptr, sy.k_ptr);
    UP(D.k_fpos, sy.k_fpos);
    UP(D.k_wslot, sy.k_wslot);
    UP(D.k_diag, sy.k_diag);
    UP(D.kc_ptr, sy.kc_ptr);
    UP(D.kc_a, sy.kc_a);
    UP(D.kc_b, sy.kc_b);
    UP(D.kc_r, sy.kc_r);
    AL(D.x0, st.nx);
    AL(D.zF, st.H);
    AL(D.uprev, st.nu);
    AL(D.y, D.n); AL(D.s, D.ml); AL(D.om, D.ml); AL(D.be, D.ml); AL(D.zl, D.n); AL(D.zu, D.n);
    AL(D.c, D.mc); AL(D.d, D.md); AL(D.jv, D.nnzj); AL(D.wv, D.nnzw); AL(D.grad, D.n); AL(D.fterm, D.n);
    AL(D.gtw, D.n); AL(D.sig, D.n); AL(D.rhs, D.n); AL(D.dy, D.n); AL(D.xp, D.n);
    AL(D.Q, D.ml); AL(D.r2, D.ml); AL(D.r4, D.ml); AL(D.qeff, D.m); AL(D.vcomb, D.m);
    AL(D.ds, D.ml); AL(D.dom, D.ml); AL(D.dbe, D.ml); AL(D.dzl, D.n); AL(D.dzu, D.n);
    AL(D.yt, D.n); AL(D.st, D.ml);
    AL(D.kv, D.nnzk); AL(D.L, sy.stored_l); AL(D.U, sy.stored_u); AL(D.uvec, sy.stored_uv);
    AL(D.fail, 1);
    AL(D.adj_rhs, D.n);
    AL(D.adj_w, D.n);
    AL(D.adj_out, st.nx + 4 + st.H);
    D.part_blocks = nblocks((int64_t)D.n + D.ml + D.m);
    AL(D.part, (size_t)kMaxQ * D.part_blocks);
    AL(D.scal, kMaxQ);
    if (!D.front_in_lds) {
        D.gstride = (int64_t)sy.max_front * (sy.max_front | 1);
        AL(D.gscratch, (size_t)D.gstride * max_groups);
    }
#undef UP
#undef AL
    e = hipHostMalloc((void**)&D.hscal, kMaxQ * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        err = std::string("hipHostMalloc: ") + hipGetErrorString(e);
        return fail_cleanup(NMPC_ERR_HIP);
    }
    e = hipHostMalloc((void**)&D.hfail, sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) {
        err = std::string("hipHostMalloc: ") + hipGetErrorString(e);
        return fail_cleanup(NMPC_ERR_HIP);
    }
    for (auto& evv : D.ev) {
        e = hipEventCreate(&evv);
        if (e != hipSuccess) {
            err = std::string("hipEventCreate: ") + hipGetErrorString(e);
            return fail_cleanup(NMPC_ERR_HIP);
        }
    }
    D.vec.n = D.n;
    D.vec.mc = D.mc;
    D.vec.md = D.md;
    D.vec.ml = D.ml;
    D.vec.lb = D.lb;
    D.vec.ub = D.ub;
    D.vec.gamma = 1e-9;
    D.S.sn_ptr = D.sn_ptr;
    D.S.rows_ptr = D.rows_ptr;
    D.S.rows = D.rows;
    D.S.child_ptr = D.child_ptr;
    D.S.child_list = D.child_list;
    D.S.l_off = D.l_off;
    D.S.u_off = D.u_off;
    D.S.uv_off = D.uv_off;
    D.S.rel_off = D.rel_off;
    D.S.rel = D.rel;
    D.S.k_ptr = D.k_ptr;
    D.S.k_fpos = D.k_fpos;
    std::string e2;
    nmpc_status rc = device_set_parameters(p, e2);
    if (rc != NMPC_OK) {
        err = e2;
        return fail_cleanup(rc);
    }
    return NMPC_OK;
}

nmpc_status device_set_parameters(Problem& p, std::string& err) {
    Device& D = *p.dev;
    HIP_TRY(hipMemcpyAsync(D.x0, p.x0.data(), p.x0.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipMemcpyAsync(D.zF, p.traj.data(), p.traj.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipMemcpyAsync(D.uprev, p.u_prev.data(), p.u_prev.size() * sizeof(double), hipMemcpyHostToDevice,
                           D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    D.dc.xD = p.setpoint.size() > 0 ? p.setpoint[0] : 0.0;
    D.dc.xB = p.setpoint.size() > 1 ? p.setpoint[1] : 0.0;
    return NMPC_OK;
}

// ---- building blocks used by the driver ----------------------------------------
namespace {

void eval(Device& D, bool full, const double* y) {
    launch_eval_distill(full, D.dd, D.dc, y, D.x0, D.zF, D.uprev, D.om, D.jptr, D.mc, D.c, D.d, D.jv, D.wv,
                        D.grad, D.fterm, D.stream);
}

Ops make_ops(std::initializer_list<int> l) {
    Ops o{};
    o.q = 0;
    for (int v : l) o.op[o.q++] = v;
    return o;
}

const Ops kOpsA = make_ops({kSum, kMax, kMax, kMax, kMax, kMin, kMax, kMin, kMax, kMin, kSum});
const Ops kOpsE = make_ops({kMin, kMin, kMax, kSum, kSum, kSum, kSum, kSum, kSum, kSum, kSum});
const Ops kOpsT = make_ops({kSum, kSum, kSum, kSum, kSum, kSum});

hipError_t fetch_scalars(Device& D, int q) {
    hipError_t e = hipMemcpyAsync(D.hscal, D.scal, q * sizeof(double), hipMemcpyDeviceToHost, D.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(D.stream);
}

void phaseA(Device& D) {
    const int nb = nblocks((int64_t)D.n + D.ml);
    hipLaunchKernelGGL(k_phaseA, dim3(nb), dim3(kBlock), 0, D.stream, D.vec, D.y, D.s, D.om, D.be, D.zl, D.zu,
                       D.grad, D.fterm, D.c, D.d, D.jv, D.jt_ptr, D.jt_slot, D.jt_row, D.gtw, D.part, kOpsA);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, D.stream, D.part, nb, kOpsA, D.scal);
}

void prep_and_assemble(Device& D, double mu) {
    hipLaunchKernelGGL(k_rows_prep, dim3(nblocks(D.m)), dim3(kBlock), 0, D.stream, D.vec, mu, D.s, D.om, D.be,
                       D.c, D.d, D.Q, D.r2, D.r4, D.qeff, D.vcomb);
    hipLaunchKernelGGL(k_var_prep, dim3(nblocks(D.n)), dim3(kBlock), 0, D.stream, D.vec, mu, D.y, D.zl, D.zu,
                       D.grad, D.gtw, D.jv, D.jt_ptr, D.jt_slot, D.jt_row, D.vcomb, D.sig, D.rhs);
    hipLaunchKernelGGL(k_assemble, dim3(nblocks(D.nnzk)), dim3(kBlock), 0, D.stream, D.nnzk, D.k_wslot, D.k_diag,
                       D.kc_ptr, D.kc_a, D.kc_b, D.kc_r, D.wv, D.sig, D.jv, D.qeff, D.kv);
}

enum Phase { kPhEval = 0, kPhAssemble = 1, kPhFactor = 2, kPhSolve = 3, kPhSearch = 4 };

struct Timer {
    Device* D;
    bool on;
    double ms[5] = {0, 0, 0, 0, 0};
    void begin(int ph) {
        if (on) (void)hipEventRecord(D->ev[2 * ph], D->stream);
    }
    void end(int ph) {
        if (on) (void)hipEventRecord(D->ev[2 * ph + 1], D->stream);
    }
    // call once the stream has passed end(ph)
    void collect(int ph) {
        if (!on) return;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, D->ev[2 * ph], D->ev[2 * ph + 1]) == hipSuccess) ms[ph] += t;
    }
};

// NumCholesky (eq. 20) of kv + eta I; returns the failure flag.
hipError_t factor(Device& D, double eta, int& failed, Timer* tm = nullptr, int* launches = nullptr) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, D.stream, D.fail);
    hipError_t e = hipSuccess;
    if (tm) tm->begin(kPhFactor);
    for (const auto& Lc : D.fwd_launches)
        launch_factor_groups(D.front_in_lds, D.sched_nodes, D.sched_gptr + Lc.gptr_off, Lc.groups, Lc.lds_factor, D.S,
                             D.kv, eta, D.L, D.U, D.fail, D.gscratch, D.gstride, D.stream);
    if (tm) tm->end(kPhFactor);
    if (launches) *launches += (int)D.fwd_launches.size();
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(D.hfail, D.fail, sizeof(int), hipMemcpyDeviceToHost, D.stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(D.stream);
    if (tm) tm->collect(kPhFactor);
    failed = *D.hfail;
    return e;
}

// Solve with the current factor: b (original order) -> x (original order).
void solve(Device& D, const double* b, double* x) {
    for (const auto& Lc : D.fwd_launches)
        launch_fwd_groups(D.sched_nodes, D.sched_gptr + Lc.gptr_off, Lc.groups, Lc.lds_solve, D.S, D.L, D.uvec, b,
                          D.perm, D.xp, D.stream);
    for (const auto& Lc : D.bwd_launches)
        launch_bwd_groups(D.sched_nodes, D.sched_gptr + Lc.gptr_off, Lc.groups, Lc.lds_solve, D.S, D.L, D.xp, D.perm,
                          x, D.stream);
}

}  // namespace

// ---- Algorithm 2 -------------------------------------------------------------------
nmpc_status device_solve(Problem& p, int warm, const nmpc_options& o, nmpc_result& r, std::string& err) {
    Device& D = *p.dev;
    D.vec.gamma = o.gamma;
    D.adj_ready = false;
    r = nmpc_result{};
    double mu = warm ? o.mu0_warm : o.mu0_cold;
    if (!warm) {
        // initial guess: every stage holds the measured state and the last control
        std::vector<double> yg(D.n);
        const int nx = p.st.nx, nu = p.st.nu, ns = nx + nu;
        for (int k = 0; k < p.st.H; ++k) {
            for (int i = 0; i < nx; ++i) yg[k * ns + i] = p.x0[i];
            for (int i = 0; i < nu; ++i) yg[k * ns + nx + i] = p.u_prev[i];
        }
        HIP_TRY(hipMemcpyAsync(D.y, yg.data(), D.n * sizeof(double), hipMemcpyHostToDevice, D.stream));
        hipLaunchKernelGGL(k_push_bounds, dim3(nblocks(D.n)), dim3(kBlock), 0, D.stream, D.vec, o.bound_push, D.y);
        eval(D, false, D.y);
        hipLaunchKernelGGL(k_cold_duals, dim3(nblocks(std::max(D.n, D.ml))), dim3(kBlock), 0, D.stream, D.vec, mu,
                           o.slack_push, D.c, D.d, D.y, D.s, D.om, D.be, D.zl, D.zu);
        HIP_TRY(hipGetLastError());
    }
    double nu = 1.0, eta_last = 0.0, eta = 0.0, E0 = INFINITY, f = 0.0;
    int it = 0, status = NMPC_MAX_ITER;
    Timer tm{&D, o.timing != 0};
    const double eps = std::numeric_limits<double>::epsilon();
    while (true) {
        tm.begin(kPhEval);
        eval(D, true, D.y);
        phaseA(D);
        tm.end(kPhEval);
        HIP_TRY(hipGetLastError());
        HIP_TRY(fetch_scalars(D, kOpsA.q));
        tm.collect(kPhEval);
        const double* A = D.hscal;
        f = A[0];
        const double dual = A[1], sinf = A[2], prim = A[3], sbmax = A[4], sbmin = A[5];
        const double lzmax = A[6], lzmin = A[7], uzmax = A[8], uzmin = A[9];
        if (A[10] > 0.0 || !std::isfinite(f)) {
            status = NMPC_NONFINITE;
            break;
        }
        auto Emu = [&](double m_) {
            double e = std::max(std::max(dual, sinf), std::max(prim, std::max(sbmax - m_, m_ - sbmin)));
            if (lzmax > -INFINITY) e = std::max(e, std::max(lzmax - m_, m_ - lzmin));
            if (uzmax > -INFINITY) e = std::max(e, std::max(uzmax - m_, m_ - uzmin));
            return e;
        };
        E0 = Emu(0.0);
        if (E0 <= o.tol) {
            status = NMPC_OK;
            break;
        }
        if (it >= o.max_iter) {
            status = NMPC_MAX_ITER;
            break;
        }
        double em = Emu(mu);
        while (em <= o.kappa_eps * mu && mu > o.mu_min) {
            mu = std::max(o.mu_min, std::min(o.kappa_mu * mu, std::pow(mu, o.theta_mu)));
            em = Emu(mu);
        }
        const double tau = std::max(o.tau_min, 1.0 - mu);
        tm.begin(kPhAssemble);
        prep_and_assemble(D, mu);
        tm.end(kPhAssemble);
        HIP_TRY(hipGetLastError());
        int failed = 0;
        eta = 0.0;
        HIP_TRY(factor(D, 0.0, failed, &tm, &r.factor_launches));
        tm.collect(kPhAssemble);
        r.factorizations++;
        if (failed) {
            eta = eta_last == 0.0 ? o.eta_first : std::max(o.eta_min, o.km * eta_last);
            bool ok = false;
            while (true) {
                HIP_TRY(factor(D, eta, failed, &tm, &r.factor_launches));
                r.factorizations++;
                if (!failed) {
                    ok = true;
                    break;
                }
                eta *= eta_last == 0.0 ? o.kp_first : o.kp;
                if (eta > o.eta_max) break;
            }
            if (!ok) {
                status = NMPC_REG_FAIL;
                break;
            }
            eta_last = eta;
        }
        tm.begin(kPhSolve);
        solve(D, D.rhs, D.dy);
        tm.end(kPhSolve);
        const int nbE = nblocks((int64_t)D.m + D.n);
        hipLaunchKernelGGL(k_phaseE, dim3(nbE), dim3(kBlock), 0, D.stream, D.vec, mu, tau, D.y, D.s, D.om, D.be,
                           D.zl, D.zu, D.grad, D.dy, D.Q, D.r2, D.r4, D.jv, D.jptr, D.jcol, D.ds, D.dom, D.dbe,
                           D.dzl, D.dzu, D.part, kOpsE);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, D.stream, D.part, nbE, kOpsE, D.scal);
        HIP_TRY(hipGetLastError());
        HIP_TRY(fetch_scalars(D, kOpsE.q));
        tm.collect(kPhSolve);
        const double* E = D.hscal;
        const double amax = std::min(1.0, E[0]);
        const double adu = std::min(1.0, E[1]);
        nu = std::max(nu, E[2] + 1.0);
        const double gfdy = E[3], dsos = E[4], dyogl = E[5], dyogu = E[6], r4l1 = E[7];
        const double lns = E[8], lngl = E[9], lngu = E[10];
        const double phi0 = f - mu * lns - mu * lngl - mu * lngu + nu * r4l1;
        const double dphi = gfdy - mu * dsos - mu * dyogl + mu * dyogu - nu * r4l1;
        double alpha = std::min(amax, adu);
        bool accepted = false;
        const int nbT = nblocks((int64_t)D.n + D.ml);
        for (int tr = 1; tr <= o.ls_max; ++tr) {
            r.ls_trials++;
            tm.begin(kPhSearch);
            hipLaunchKernelGGL(k_trial_point, dim3(nblocks(std::max(D.n, D.ml))), dim3(kBlock), 0, D.stream, D.n,
                               D.ml, alpha, D.y, D.dy, D.s, D.ds, D.yt, D.st);
            eval(D, false, D.yt);
            hipLaunchKernelGGL(k_phaseT, dim3(nbT), dim3(kBlock), 0, D.stream, D.vec, D.yt, D.st, D.fterm, D.c, D.d,
                               D.part, kOpsT);
            hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, D.stream, D.part, nbT, kOpsT, D.scal);
            tm.end(kPhSearch);
            HIP_TRY(hipGetLastError());
            HIP_TRY(fetch_scalars(D, kOpsT.q));
            tm.collect(kPhSearch);
            const double* T = D.hscal;
            const double phit = T[0] - mu * T[1] - mu * T[2] - mu * T[3] + nu * T[4];
            if (T[5] == 0.0 && std::isfinite(phit) &&
                phit <= phi0 + o.armijo * alpha * dphi + 10.0 * eps * std::fabs(phi0)) {
                accepted = true;
                break;
            }
            alpha *= 0.5;
        }
        if (!accepted) {
            status = NMPC_LINESEARCH_FAIL;
            break;
        }
        hipLaunchKernelGGL(k_update, dim3(nblocks(std::max(D.n, D.ml))), dim3(kBlock), 0, D.stream, D.vec, alpha,
                           mu, o.kappa_sigma, D.y, D.s, D.om, D.be, D.zl, D.zu, D.dy, D.ds, D.dom, D.dbe, D.dzl,
                           D.dzu);
        HIP_TRY(hipGetLastError());
        ++it;
    }
    HIP_TRY(hipStreamSynchronize(D.stream));
    r.status = status;
    r.iters = it;
    r.mu = mu;
    r.eta = eta;
    r.E0 = E0;
    r.objective = f;
    r.ms_eval = tm.ms[kPhEval];
    r.ms_assemble = tm.ms[kPhAssemble];
    r.ms_factor = tm.ms[kPhFactor];
    r.ms_solve = tm.ms[kPhSolve];
    r.ms_linesearch = tm.ms[kPhSearch];
    return status;
}

nmpc_status device_get_iterate(const Problem& p, double* y, double* s, double* om, double* be, double* zl,
                               double* zu, std::string& err) {
    const Device& D = *p.dev;
    HIP_TRY(hipMemcpy(y, D.y, D.n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s, D.s, D.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(om, D.om, D.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(be, D.be, D.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(zl, D.zl, D.n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(zu, D.zu, D.n * sizeof(double), hipMemcpyDeviceToHost));
    return NMPC_OK;
}

nmpc_status device_set_iterate(Problem& p, const double* y, const double* s, const double* om, const double* be,
                               const double* zl, const double* zu, std::string& err) {
    Device& D = *p.dev;
    D.adj_ready = false;
    HIP_TRY(hipMemcpy(D.y, y, D.n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D.s, s, D.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D.om, om, D.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D.be, be, D.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D.zl, zl, D.n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(D.zu, zu, D.n * sizeof(double), hipMemcpyHostToDevice));
    return NMPC_OK;
}

nmpc_status device_eval(Problem& p, const double* y, const double* lam, const double* lam_d, double* f,
                        double* grad, double* c, double* d, double* jv, double* wv, std::string& err) {
    Device& D = *p.dev;
    // stage the multipliers as a lifted omega: omega+ = lam, omega- = 0, omega_d = lam_d
    std::vector<double> om(D.ml, 0.0);
    for (int r = 0; r < D.mc; ++r) om[r] = lam[r];
    for (int r = 0; r < D.md; ++r) om[2 * D.mc + r] = lam_d[r];
    HIP_TRY(hipMemcpyAsync(D.yt, y, D.n * sizeof(double), hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipMemcpyAsync(D.dom, om.data(), D.ml * sizeof(double), hipMemcpyHostToDevice, D.stream));
    launch_eval_distill(true, D.dd, D.dc, D.yt, D.x0, D.zF, D.uprev, D.dom, D.jptr, D.mc, D.c, D.d, D.jv, D.wv,
                        D.grad, D.fterm, D.stream);
    HIP_TRY(hipGetLastError());
    std::vector<double> ft(D.n);
    HIP_TRY(hipMemcpyAsync(ft.data(), D.fterm, D.n * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (grad) HIP_TRY(hipMemcpyAsync(grad, D.grad, D.n * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (c) HIP_TRY(hipMemcpyAsync(c, D.c, D.mc * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (d && D.md) HIP_TRY(hipMemcpyAsync(d, D.d, D.md * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (jv) HIP_TRY(hipMemcpyAsync(jv, D.jv, D.nnzj * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (wv) HIP_TRY(hipMemcpyAsync(wv, D.wv, D.nnzw * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    if (f) {
        double acc = 0.0;
        for (double v : ft) acc += v;
        *f = acc;
    }
    return NMPC_OK;
}

nmpc_status device_factor(Problem& p, const double* kv, double eta, int32_t* ok, double* lv, std::string& err) {
    Device& D = *p.dev;
    HIP_TRY(hipMemcpyAsync(D.kv, kv, D.nnzk * sizeof(double), hipMemcpyHostToDevice, D.stream));
    int failed = 0;
    HIP_TRY(factor(D, eta, failed));
    *ok = failed ? 0 : 1;
    if (lv) HIP_TRY(hipMemcpy(lv, D.L, p.sym.stored_l * sizeof(double), hipMemcpyDeviceToHost));
    return NMPC_OK;
}

nmpc_status device_linear_solve(Problem& p, const double* b, double* x, std::string& err) {
    Device& D = *p.dev;
    HIP_TRY(hipMemcpyAsync(D.yt, b, D.n * sizeof(double), hipMemcpyHostToDevice, D.stream));
    solve(D, D.yt, D.dzl);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(x, D.dzl, D.n * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    return NMPC_OK;
}

nmpc_status device_assemble(Problem& p, double mu, double* kv, double* rhs, std::string& err) {
    Device& D = *p.dev;
    eval(D, true, D.y);
    phaseA(D);
    prep_and_assemble(D, mu);
    HIP_TRY(hipGetLastError());
    if (kv) HIP_TRY(hipMemcpyAsync(kv, D.kv, D.nnzk * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    if (rhs) HIP_TRY(hipMemcpyAsync(rhs, D.rhs, D.n * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    return NMPC_OK;
}

}  // namespace nmpc

namespace nmpc {

void device_invalidate_adjoint(Problem& p) {
    if (p.dev) p.dev->adj_ready = false;
}

namespace {

// Assemble and factor K at the handle's iterate (inertia correction as in the solve).
nmpc_status adjoint_prepare(Problem& p, std::string& err) {
    Device& D = *p.dev;
    if (D.adj_ready) return NMPC_OK;
    eval(D, true, D.y);
    phaseA(D);
    prep_and_assemble(D, 1.0);   // mu only enters r2, which the sensitivities do not use
    HIP_TRY(hipGetLastError());
    int failed = 0;
    double eta = 0.0;
    HIP_TRY(factor(D, 0.0, failed));
    if (failed) {
        nmpc_options o;
        nmpc_default_options(&o);
        eta = o.eta_first;
        while (true) {
            HIP_TRY(factor(D, eta, failed));
            if (!failed) break;
            eta *= o.kp_first;
            if (eta > o.eta_max) {
                err = "adjoint: the condensed matrix at the solution could not be factored";
                return NMPC_ERR_INVALID_ARG;
            }
        }
    }
    D.adj_eta = eta;
    D.adj_ready = true;
    return NMPC_OK;
}

nmpc_status adjoint_apply(Problem& p, const double* seed_u1, double seed_obj, std::vector<double>& out,
                          std::string& err) {
    Device& D = *p.dev;
    const Structure& st = p.st;
    if (st.nu > kMaxSeed) {
        err = "adjoint: too many controls per stage";
        return NMPC_ERR_UNSUPPORTED;
    }
    Seed sd{};
    for (int j = 0; j < st.nu; ++j) sd.u[j] = seed_u1[j];
    hipLaunchKernelGGL(k_adj_seed, dim3(nblocks(D.n)), dim3(kBlock), 0, D.stream, D.n, st.nx, st.nu, D.grad,
                       seed_obj, sd, D.adj_rhs);
    solve(D, D.adj_rhs, D.adj_w);
    hipLaunchKernelGGL(k_adj_gather_distill, dim3(1), dim3(kBlock), 0, D.stream, D.dd, D.dc, D.y, D.uprev, D.adj_w,
                       D.jv, D.jptr, D.jcol, D.qeff, seed_obj, D.adj_out);
    HIP_TRY(hipGetLastError());
    out.resize(st.nx + 4 + st.H);
    HIP_TRY(hipMemcpyAsync(out.data(), D.adj_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    return NMPC_OK;
}

}  // namespace

nmpc_status device_adjoint(Problem& p, const double* seed_u1, double seed_obj, double* gx0, double* gsp,
                           double* gtraj, double* gup, std::string& err) {
    nmpc_status rc = adjoint_prepare(p, err);
    if (rc != NMPC_OK) return rc;
    std::vector<double> out;
    rc = adjoint_apply(p, seed_u1, seed_obj, out, err);
    if (rc != NMPC_OK) return rc;
    const Structure& st = p.st;
    if (gx0) std::copy(out.begin(), out.begin() + st.nx, gx0);
    if (gsp) std::copy(out.begin() + st.nx, out.begin() + st.nx + 2, gsp);
    if (gtraj) std::copy(out.begin() + st.nx + 2, out.begin() + st.nx + 2 + st.H, gtraj);
    if (gup) std::copy(out.begin() + st.nx + 2 + st.H, out.begin() + st.nx + 4 + st.H, gup);
    return p.dev->adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

nmpc_status device_jacobian_u1_x0(Problem& p, double* jac, std::string& err) {
    nmpc_status rc = adjoint_prepare(p, err);
    if (rc != NMPC_OK) return rc;
    const Structure& st = p.st;
    std::vector<double> seed(st.nu, 0.0), out;
    for (int j = 0; j < st.nu; ++j) {
        std::fill(seed.begin(), seed.end(), 0.0);
        seed[j] = 1.0;
        rc = adjoint_apply(p, seed.data(), 0.0, out, err);
        if (rc != NMPC_OK) return rc;
        std::copy(out.begin(), out.begin() + st.nx, jac + (size_t)j * st.nx);
    }
    return p.dev->adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

}  // namespace nmpc
