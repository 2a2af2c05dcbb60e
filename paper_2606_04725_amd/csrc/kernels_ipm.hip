// Interior-point vector kernels and per-instance decisions of Algorithm 2.
//
// Every vector kernel maps its blocks to instances through an index space
// (binst / bfirst) and returns at once for an instance whose control block is
// not in the kernel's phase, so one launch serves a batch and a pass of the
// method can be replayed as a graph with converged instances idle.
//
// Reductions are two-level and deterministic: each block reduces its slice of
// one instance in a fixed tree order into that instance's partial buffer, then
// the instance's decision block reduces the partials in block order and takes
// the method's scalar decisions (barrier update, regularization, step
// acceptance) on the device.
#include <cmath>

#include "kernels.h"

namespace nmpc {

namespace {

enum Op : int { kSum = 0, kMax = 1, kMin = 2 };

__device__ inline double combine(int op, double a, double b) {
    return op == kSum ? a + b : (op == kMax ? fmax(a, b) : fmin(a, b));
}

__device__ inline double ident(int op) {
    return op == kSum ? 0.0 : (op == kMax ? -INFINITY : INFINITY);
}

struct Ops {
    int q;
    int op[kMaxQ];
};

constexpr Ops kOpsA{11, {kSum, kMax, kMax, kMax, kMax, kMin, kMax, kMin, kMax, kMin, kSum}};
constexpr Ops kOpsE{11, {kMin, kMin, kMax, kSum, kSum, kSum, kSum, kSum, kSum, kSum, kSum}};
constexpr Ops kOpsT{6, {kSum, kSum, kSum, kSum, kSum, kSum}};

constexpr int kWaves = kBlock / 64;

// Butterfly reduction across the 64 lanes of a wave (fixed pattern).
__device__ inline double wave_reduce(double v, int op) {
    for (int off = 32; off > 0; off >>= 1) v = combine(op, v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce every quantity over the block (waves, then the per-wave results in
// wave order); thread q returns quantity q's block result in out (q < ops.q).
// The butterfly steps of all quantities go level by level, so each level's
// lane exchanges are in flight together (per quantity the same steps as
// wave_reduce).
__device__ __attribute__((always_inline)) inline double block_reduce(const double* v, const Ops& ops, double* sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double r[kMaxQ];
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) r[q] = q < ops.q ? v[q] : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double x[kMaxQ];
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q)
            if (q < ops.q) x[q] = __shfl_xor(r[q], off, 64);
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q)
            if (q < ops.q) r[q] = combine(ops.op[q], r[q], x[q]);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q)
            if (q < ops.q) sh[q * kWaves + wv] = r[q];
    }
    __syncthreads();
    double acc = 0.0;
    if ((int)threadIdx.x < ops.q) {
        const int q = threadIdx.x;
        acc = sh[q * kWaves];
        for (int w = 1; w < kWaves; ++w) acc = combine(ops.op[q], acc, sh[q * kWaves + w]);
    }
    return acc;
}

// Block partials of one instance: part[q * nb + lb].
__device__ __attribute__((always_inline)) inline void store_partials(const double* v, const Ops& ops, double* part, int nb, int lb, double* sh) {
    const double r = block_reduce(v, ops, sh);
    if ((int)threadIdx.x < ops.q) part[(int64_t)threadIdx.x * nb + lb] = r;
}

// Decision block of one instance: reduce its nb partials in block order; the
// totals land in tot[0 .. ops.q) (shared memory) for thread 0.
__device__ __attribute__((always_inline)) inline void finalize_partials(const double* part, int nb, const Ops& ops, double* sh, double* tot) {
    double v[kMaxQ];
#pragma unroll
    for (int q = 0; q < kMaxQ; ++q) v[q] = q < ops.q ? ident(ops.op[q]) : 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {   // per quantity in block order; the loads go together
        double x[kMaxQ];
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q)
            if (q < ops.q) x[q] = part[(int64_t)q * nb + b];
#pragma unroll
        for (int q = 0; q < kMaxQ; ++q)
            if (q < ops.q) v[q] = combine(ops.op[q], v[q], x[q]);
    }
    const double r = block_reduce(v, ops, sh);
    if ((int)threadIdx.x < ops.q) tot[threadIdx.x] = r;
    __syncthreads();
}

// acc + sum of term(index(e)) over the entries e in [e0, e1), added in entry
// order; a batch of kGather entries loads its indices, then its values, before
// the first addition (past e1 a batch repeats entry e0, whose terms it drops).
constexpr int kGather = 8;
template <class Index, class Term>
__device__ __attribute__((always_inline)) inline double gather_sum(int e0, int e1, double acc, Index index, Term term) {
    using Ix = decltype(index(0));
    for (int eb = e0; eb < e1; eb += kGather) {
        Ix ix[kGather];
#pragma unroll
        for (int u = 0; u < kGather; ++u) ix[u] = index(eb + u < e1 ? eb + u : e0);
        double t[kGather];
#pragma unroll
        for (int u = 0; u < kGather; ++u) t[u] = term(ix[u]);
#pragma unroll
        for (int u = 0; u < kGather; ++u)
            if (eb + u < e1) acc += t[u];
    }
    return acc;
}

__device__ inline bool hasL(const InstPtrs& I, int j) { return I.lb[j] > -INFINITY; }
__device__ inline bool hasU(const InstPtrs& I, int j) { return I.ub[j] < INFINITY; }

// Lifted row r: c_r - gamma, -c_{r - mc} - gamma, or d_{r - 2 mc}; one load
// from a per-lane source (no branch, so it issues with the caller's others).
__device__ inline double lifted_g(const InstPtrs& I, double gamma, int r) {
    const bool up = r < I.mc, lo = !up && r < 2 * I.mc;
    const double* src = up || lo ? I.c : I.d;
    const double v = src[up ? r : (lo ? r - I.mc : r - 2 * I.mc)];
    return up ? v - gamma : (lo ? -v - gamma : v);
}

__device__ inline int nblocks_of(const Space& sp, int inst) { return sp.bfirst[inst + 1] - sp.bfirst[inst]; }

// ---- phase A: optimality-error ingredients at the current iterate --------------
// q: 0 f(sum) 1 dual(max) 2 |omega-beta|(max) 3 |g+s|(max) 4 sb max 5 sb min
//    6 gL zL max 7 gL zL min 8 gU zU max 9 gU zU min 10 non-finite count(sum)
__global__ void __launch_bounds__(kBlock) k_phaseA(const InstPtrs* __restrict__ Ia, Space sp, int pred) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, pred)) return;
    const double gamma = I.ctl->gamma;
    double q[11] = {0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, 0.0};
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) {
        const int j = t;
        // the variable's own values are loaded with the gather's first indices
        const double lbj = I.lb[j], ubj = I.ub[j], yj = I.y[j], zlj = I.zl[j], zuj = I.zu[j];
        const double gradj = I.grad[j], ftj = I.fterm[j];
        const double acc = gather_sum(
            I.jt_ptr[j], I.jt_ptr[j + 1], 0.0, [&](int e) { return int2{I.jt_row[e], I.jt_slot[e]}; },
            [&](int2 rs) {
                // both multipliers are loaded whatever the row's kind, so the
                // batch's loads are issued together (no branch between them)
                const int r = rs.x;
                const double a = I.om[r < I.mc ? r : I.mc + r], b = I.om[I.mc + r];
                const double lam = r < I.mc ? a - b : b;
                return I.jv[rs.y] * lam;
            });
        I.gtw[j] = acc;
        const bool hl = lbj > -INFINITY, hu = ubj < INFINITY;
        const double zl = hl ? zlj : 0.0, zu = hu ? zuj : 0.0;
        const double dual = gradj + acc - zl + zu;
        q[0] = ftj;
        q[1] = fabs(dual);
        if (hl) {
            const double p = (yj - lbj) * zl;
            q[6] = p;
            q[7] = p;
        }
        if (hu) {
            const double p = (ubj - yj) * zu;
            q[8] = p;
            q[9] = p;
        }
        if (!isfinite(ftj) || !isfinite(gradj)) q[10] = 1.0;
    } else if (t < I.n + I.ml) {
        const int r = t - I.n;
        if (I.ctl->hyk && r < 2 * I.mc) {
            // HyKKT: an equality row has no slack; its residual is c itself
            if (r < I.mc) {
                q[3] = fabs(I.c[r]);
                if (!isfinite(I.c[r])) q[10] = 1.0;
            }
        } else {
            const double g = lifted_g(I, gamma, r);
            q[2] = fabs(I.om[r] - I.be[r]);
            q[3] = fabs(g + I.s[r]);
            q[4] = I.s[r] * I.be[r];
            q[5] = q[4];
            if (!isfinite(g)) q[10] = 1.0;
        }
    }
    store_partials(q, kOpsA, I.part, nblocks_of(sp, inst), lb, sh);
}

// Optimality errors (eqs. 27-28), termination and the barrier update.
__global__ void __launch_bounds__(kBlock) k_decideA(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double A[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (c->phase != kPhA) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsA, sh, A);
    if (threadIdx.x != 0) return;
    const double f = A[0];
    c->f = f;
    const double dual = A[1], sinf = A[2], prim = A[3], sbmax = A[4], sbmin = A[5];
    const double lzmax = A[6], lzmin = A[7], uzmax = A[8], uzmin = A[9];
    if (A[10] > 0.0 || !isfinite(f)) {
        c->status = NMPC_NONFINITE;
        c->phase = kPhDone;
        return;
    }
    auto Emu = [&](double m_) {
        double e = fmax(fmax(dual, sinf), fmax(prim, fmax(sbmax - m_, m_ - sbmin)));
        if (lzmax > -INFINITY) e = fmax(e, fmax(lzmax - m_, m_ - lzmin));
        if (uzmax > -INFINITY) e = fmax(e, fmax(uzmax - m_, m_ - uzmin));
        return e;
    };
    const double E0 = Emu(0.0);
    c->E0 = E0;
    // termination: eq. (28) on E_0, or, on one fixed barrier problem, E_mu
    if ((o.fixed_mu ? Emu(c->mu) : E0) <= o.tol) {
        c->status = NMPC_OK;
        c->phase = kPhDone;
        return;
    }
    if (c->it >= o.max_iter) {
        c->status = NMPC_MAX_ITER;
        c->phase = kPhDone;
        return;
    }
    double mu = c->mu;
    double em = Emu(mu);
    while (!o.fixed_mu && em <= o.kappa_eps * mu && mu > o.mu_min) {
        mu = fmax(o.mu_min, fmin(o.kappa_mu * mu, pow(mu, o.theta_mu)));
        em = Emu(mu);
    }
    c->mu = mu;
    c->tau = fmax(o.tau_min, 1.0 - mu);
    c->eta = 0.0;
    c->fail = 0;
    c->phase = kPhB;
}

// ---- phase B: condensed system ingredients --------------------------------------
// per original row r: lifted Q, r2, r4 and their combinations
//   c row r:  qeff = Q+ + Q-,  vcomb = (Q+ r4+ - r2+) - (Q- r4- - r2-)
//   d row r:  qeff = Q,        vcomb = Q r4 - r2
__global__ void __launch_bounds__(kBlock) k_rows_prep(const InstPtrs* __restrict__ Ia, Space sp, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, pred)) return;
    const double mu = I.ctl->mu, gamma = I.ctl->gamma;
    const int r = lb * kBlock + threadIdx.x;
    if (r >= I.m) return;
    if (r < I.mc && I.ctl->hyk) {
        // HyKKT: weight hk_gamma on J_c^T J_c, right-hand side b1 + hk_gamma J_c^T b2 with b2 = -c
        const int a = r, b = I.mc + r;
        const double g = I.ctl->hk_gamma;
        I.Q[a] = 0.0; I.Q[b] = 0.0;
        I.r2[a] = 0.0; I.r2[b] = 0.0;
        I.r4[a] = I.c[r]; I.r4[b] = 0.0;
        I.qeff[r] = g;
        I.vcomb[r] = g * I.c[r];
    } else if (r < I.mc) {
        const int a = r, b = I.mc + r;
        const double Qa = I.be[a] / I.s[a], Qb = I.be[b] / I.s[b];
        const double r2a = I.om[a] - mu / I.s[a], r2b = I.om[b] - mu / I.s[b];
        const double r4a = lifted_g(I, gamma, a) + I.s[a], r4b = lifted_g(I, gamma, b) + I.s[b];
        I.Q[a] = Qa; I.Q[b] = Qb;
        I.r2[a] = r2a; I.r2[b] = r2b;
        I.r4[a] = r4a; I.r4[b] = r4b;
        I.qeff[r] = Qa + Qb;
        I.vcomb[r] = (Qa * r4a - r2a) - (Qb * r4b - r2b);
    } else {
        const int a = I.mc + r;
        const double Qa = I.be[a] / I.s[a];
        const double r2a = I.om[a] - mu / I.s[a];
        const double r4a = lifted_g(I, gamma, a) + I.s[a];
        I.Q[a] = Qa; I.r2[a] = r2a; I.r4[a] = r4a;
        I.qeff[r] = Qa;
        I.vcomb[r] = Qa * r4a - r2a;
    }
}

// per variable: Sigma, and rhs = -r1 - G^T (Q r4 - r2), r1 = grad + G^T omega - mu/gL + mu/gU
__global__ void __launch_bounds__(kBlock) k_var_prep(const InstPtrs* __restrict__ Ia, Space sp, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, pred)) return;
    const double mu = I.ctl->mu;
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n) return;
    // every load (the variable's values and the gather) before the first store
    const double lbj = I.lb[j], ubj = I.ub[j], yj = I.y[j], zlj = I.zl[j], zuj = I.zu[j];
    const double gradj = I.grad[j], gtwj = I.gtw[j];
    const double acc = gather_sum(
        I.jt_ptr[j], I.jt_ptr[j + 1], 0.0, [&](int e) { return int2{I.jt_row[e], I.jt_slot[e]}; },
        [&](int2 rs) { return I.jv[rs.y] * I.vcomb[rs.x]; });
    const bool hl = lbj > -INFINITY, hu = ubj < INFINITY;
    const double gl = hl ? yj - lbj : 1.0;
    const double gu = hu ? ubj - yj : 1.0;
    I.sig[j] = (hl ? zlj / gl : 0.0) + (hu ? zuj / gu : 0.0);
    const double r1 = gradj + gtwj - (hl ? mu / gl : 0.0) + (hu ? mu / gu : 0.0);
    I.r1v[j] = r1;
    I.rhs[j] = -r1 - acc;
}

// K slot values: W + Sigma + J^T diag(qeff) J, gathered per slot (no atomics)
__global__ void __launch_bounds__(kBlock) k_assemble(const InstPtrs* __restrict__ Ia, Space sp, int pred) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, pred)) return;
    const int64_t t = (int64_t)lb * kBlock + threadIdx.x;
    if (t >= I.nnzk) return;
    const int ws = I.k_wslot[t], dg = I.k_diag[t];
    double v = ws >= 0 ? I.wv[ws] : 0.0;
    if (dg >= 0) v += I.sig[dg];
    v = gather_sum(
        I.kc_ptr[t], I.kc_ptr[t + 1], v, [&](int e) { return int3{I.kc_a[e], I.kc_r[e], I.kc_b[e]}; },
        [&](int3 arb) { return I.jv[arb.x] * I.qeff[arb.y] * I.jv[arb.z]; });
    I.kv[t] = v;
}

// Inertia correction after a factorization attempt (eqs. 12-13): on failure the
// next eta (first from eta_last, then growing); on success the step solve.
__global__ void k_decideF(const InstPtrs* __restrict__ Ia, int ninst, DevOpts o) {
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= ninst) return;
    Ctl* c = Ia[inst].ctl;
    const int ph = c->phase;
    if (ph != kPhB && ph != kPhF) return;
    c->factorizations += 1;
    if (c->fail) {
        c->fail = 0;
        if (ph == kPhB) {
            c->eta = c->eta_last == 0.0 ? o.eta_first : fmax(o.eta_min, o.km * c->eta_last);
            c->phase = kPhF;
        } else {
            const double eta = c->eta * (c->eta_last == 0.0 ? o.kp_first : o.kp);
            c->eta = eta;
            if (eta > o.eta_max) {
                c->status = NMPC_REG_FAIL;
                c->phase = kPhDone;
            }
        }
    } else {
        if (ph == kPhF) c->eta_last = c->eta;
        c->phase = kPhS;
    }
}

__device__ inline double ftb(double v, double dv, double tau) { return dv < 0.0 ? (-tau * v) / dv : INFINITY; }

// The filter search found no acceptable point: restart the backtracking from
// the fraction-to-boundary step on the l1 merit phi + nu theta, or stop.
__device__ void filter_search_failed(Ctl* c, const DevOpts& o) {
    if (o.merit_fallback && o.ls_max > 0) {
        c->ls_merit = 1;
        c->merit_trials = 0;
        c->nu = fmax(c->nu, c->om_max + 1.0);
        c->alpha = c->amax0;
        c->phase = kPhT;
    } else {
        c->status = NMPC_LINESEARCH_FAIL;
        c->phase = kPhDone;
    }
}

// ---- phase S: remaining directions and step / merit ingredients ------------------
// q: 0 alpha_primal(min) 1 alpha_dual(min) 2 max |omega + d_omega| 3 grad.dy 4 sum ds/s
//    5 sum dy/gL 6 sum dy/gU 7 |r4|_1 8 sum ln s 9 sum ln gL 10 sum ln gU
__global__ void __launch_bounds__(kBlock) k_phaseE(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, kPhS)) return;
    const double mu = I.ctl->mu, tau = I.ctl->tau;
    double q[11] = {INFINITY, INFINITY, -INFINITY, 0, 0, 0, 0, 0, 0, 0, 0};
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.m && t < I.mc && I.ctl->hyk) {
        // HyKKT: the equality multiplier moves by the CG solution; no slack
        const int r = t, b = I.mc + r;
        const double dl = I.hk_x[r];
        I.ds[r] = 0.0; I.dom[r] = dl; I.dbe[r] = 0.0;
        I.ds[b] = 0.0; I.dom[b] = 0.0; I.dbe[b] = 0.0;
        q[2] = fabs(I.om[r] + dl);
        q[7] = fabs(I.r4[r]);
    } else if (t < I.m) {
        const int r = t;
        // the lifted rows of r: r and mc + r for an equality row, mc + r
        // otherwise; every operand of both is loaded before the row's product
        // and the first store
        const bool eq = r < I.mc;
        const int nl = eq ? 2 : 1;
        int l[2];
        l[0] = eq ? r : I.mc + r;
        l[1] = I.mc + r;
        double sl[2], Ql[2], r4[2], r2[2], be[2], om[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            sl[h] = I.s[l[h]];
            Ql[h] = I.Q[l[h]];
            r4[h] = I.r4[l[h]];
            r2[h] = I.r2[l[h]];
            be[h] = I.be[l[h]];
            om[h] = I.om[l[h]];
        }
        double jdy = 0.0;
        for (int p = I.jptr[r]; p < I.jptr[r + 1]; ++p) jdy += I.jv[p] * I.dy[I.jcol[p]];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nl) break;
            const double sgn = (eq && h == 1) ? -1.0 : 1.0;
            const double dsl = -r4[h] - sgn * jdy;
            const double doml = -r2[h] - Ql[h] * dsl;
            const double dbel = mu / sl[h] - be[h] - Ql[h] * dsl;
            I.ds[l[h]] = dsl;
            I.dom[l[h]] = doml;
            I.dbe[l[h]] = dbel;
            q[0] = fmin(q[0], ftb(sl[h], dsl, tau));
            q[2] = fmax(q[2], fabs(om[h] + doml));
            q[1] = fmin(q[1], ftb(be[h], dbel, tau));
            q[4] += dsl / sl[h];
            q[7] += fabs(r4[h]);
            q[8] += log(sl[h]);
        }
    } else if (t < I.m + I.n) {
        const int j = t - I.m;
        const bool hl = hasL(I, j), hu = hasU(I, j);
        const double gl = hl ? I.y[j] - I.lb[j] : 1.0;
        const double gu = hu ? I.ub[j] - I.y[j] : 1.0;
        const double dyj = I.dy[j];
        const double zlj = I.zl[j], zuj = I.zu[j];
        const double zl = hl ? zlj : 0.0, zu = hu ? zuj : 0.0;
        const double dzlj = hl ? mu / gl - zl - (zl / gl) * dyj : 0.0;
        const double dzuj = hu ? mu / gu - zu + (zu / gu) * dyj : 0.0;
        I.dzl[j] = dzlj;
        I.dzu[j] = dzuj;
        q[3] = I.grad[j] * dyj;
        if (hl) {
            q[0] = fmin(q[0], ftb(gl, dyj, tau));
            q[1] = fmin(q[1], ftb(zl, dzlj, tau));
            q[5] = dyj / gl;
            q[9] = log(gl);
        }
        if (hu) {
            q[0] = fmin(q[0], ftb(gu, -dyj, tau));
            q[1] = fmin(q[1], ftb(zu, dzuj, tau));
            q[6] = dyj / gu;
            q[10] = log(gu);
        }
    }
    store_partials(q, kOpsE, I.part, nblocks_of(sp, inst), lb, sh);
}

// Step bound (eq. 26) and the filter line search's quantities at the iterate:
// violation theta = |g^l + s|_1, barrier objective phi, its directional
// derivative, the minimal step; the filter is reset when mu has changed and
// the theta bounds are fixed at the first iteration of a solve.
__global__ void __launch_bounds__(kBlock) k_decideE(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double E[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (c->phase != kPhS) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsE, sh, E);
    if (threadIdx.x != 0) return;
    const double mu = c->mu;
    const double amax = fmin(1.0, E[0]);
    const double adu = fmin(1.0, E[1]);
    const double gfdy = E[3], dsos = E[4], dyogl = E[5], dyogu = E[6], theta = E[7];
    const double lns = E[8], lngl = E[9], lngu = E[10];
    const double phi0 = c->f - mu * lns - mu * lngl - mu * lngu;
    const double dphi = gfdy - mu * dsos - mu * dyogl + mu * dyogu;
    if (c->it == 0) {
        c->theta_max = o.theta_max_fact * fmax(1.0, theta);
        c->theta_min = o.theta_min_fact * fmax(1.0, theta);
    }
    if (!(mu == c->filter_mu)) {
        c->filter_n = 0;
        c->filter_mu = mu;
    }
    double amin;
    if (dphi < 0.0) {
        amin = fmin(o.g_theta, o.g_phi * theta / (-dphi));
        if (theta <= c->theta_min) amin = fmin(amin, o.delta * pow(theta, o.s_theta) / pow(-dphi, o.s_phi));
    } else {
        amin = o.g_theta;
    }
    amin *= o.amin_frac;
    const double alpha = fmin(amax, adu);
    c->theta = theta;
    c->phi0 = phi0;
    c->dphi = dphi;
    c->amin = amin;
    c->alpha = alpha;
    c->trials = 0;
    c->use_soc = 0;
    c->amax0 = alpha;
    c->om_max = E[2];
    c->ls_merit = 0;
    if (alpha >= amin && o.ls_max > 0) {
        c->phase = kPhT;
    } else {
        filter_search_failed(c, o);
    }
}

__global__ void __launch_bounds__(kBlock) k_trial_point(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, kPhT)) return;
    const double alpha = I.ctl->alpha;
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) I.yt[t] = I.y[t] + alpha * I.dy[t];
    if (t < I.ml) I.st[t] = I.s[t] + alpha * I.ds[t];
}

// merit ingredients at the trial point
// q: 0 f(sum) 1 sum ln s 2 sum ln gL 3 sum ln gU 4 |g+s|_1 5 non-finite count
__global__ void __launch_bounds__(kBlock) k_phaseT(const InstPtrs* __restrict__ Ia, Space sp, int pred) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, pred)) return;
    const double gamma = I.ctl->gamma;
    double q[6] = {0, 0, 0, 0, 0, 0};
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) {
        const int j = t;
        q[0] = I.fterm[j];
        if (hasL(I, j)) q[2] = log(I.yt[j] - I.lb[j]);
        if (hasU(I, j)) q[3] = log(I.ub[j] - I.yt[j]);
        if (!isfinite(I.fterm[j])) q[5] = 1.0;
    } else if (t < I.n + I.ml) {
        const int r = t - I.n;
        if (I.ctl->hyk && r < 2 * I.mc) {
            if (r < I.mc) {
                q[4] = fabs(I.c[r]);
                if (!isfinite(I.c[r])) q[5] = 1.0;
            }
        } else {
            const double g = lifted_g(I, gamma, r);
            q[1] = log(I.st[r]);
            q[4] = fabs(g + I.st[r]);
            if (!isfinite(g)) q[5] = 1.0;
        }
    }
    store_partials(q, kOpsT, I.part, nblocks_of(sp, inst), lb, sh);
}

// Filter test of a trial point (violation tht, barrier objective pht) for a
// step of length alpha along the Newton direction: filter acceptability, then
// Armijo when the switching condition holds, sufficient decrease of theta or
// phi otherwise (then the filter takes ((1 - g_theta) theta, phi - g_phi theta),
// dropping the entries it dominates, the oldest one when it is full).
__device__ bool filter_accepts(const InstPtrs& I, Ctl* c, const DevOpts& o, double tht, double pht, bool finite,
                               double alpha) {
    const double phi0 = c->phi0, theta = c->theta, dphi = c->dphi;
    double* F = I.filter;
    const int nf = c->filter_n;
    bool ok = finite && isfinite(pht) && isfinite(tht) && tht < c->theta_max;
    for (int e = 0; ok && e < nf; ++e)
        if (!(tht < F[2 * e] || pht < F[2 * e + 1])) ok = false;
    if (!ok) return false;
    const bool switching = dphi < 0.0 && theta <= c->theta_min &&
                           alpha * pow(-dphi, o.s_phi) > o.delta * pow(theta, o.s_theta);
    if (switching) {
        const double eps = 2.220446049250313e-16;
        return pht <= phi0 + o.armijo * alpha * dphi + 10.0 * eps * fabs(phi0);
    }
    if (!(tht <= (1.0 - o.g_theta) * theta || pht <= phi0 - o.g_phi * theta)) return false;
    const double et = (1.0 - o.g_theta) * theta, ep = phi0 - o.g_phi * theta;
    int w = 0;
    for (int e = 0; e < nf; ++e) {
        const double ft = F[2 * e], fp = F[2 * e + 1];
        if (ft >= et && fp >= ep) continue;
        F[2 * w] = ft;
        F[2 * w + 1] = fp;
        ++w;
    }
    if (w >= o.filter_cap) {   // full: drop the oldest entry
        for (int e = 1; e < w; ++e) {
            F[2 * (e - 1)] = F[2 * e];
            F[2 * (e - 1) + 1] = F[2 * e + 1];
        }
        --w;
    }
    F[2 * w] = et;
    F[2 * w + 1] = ep;
    c->filter_n = w + 1;
    return true;
}

// Trial point verdict; a rejected first trial that does not reduce theta goes
// to the second-order corrections, otherwise alpha is halved, and the filter
// search ends when alpha falls below the minimal step or the trial budget is
// spent.  In the merit search (after a failed filter search) the test is
// Armijo on phi + nu theta, with its own budget of trials.
__global__ void __launch_bounds__(kBlock) k_decideT(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double T[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (c->phase != kPhT) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsT, sh, T);
    if (threadIdx.x != 0) return;
    const double mu = c->mu, alpha = c->alpha;
    c->ls_trials += 1;
    c->trials += 1;
    const double pht = T[0] - mu * T[1] - mu * T[2] - mu * T[3];
    const double tht = T[4];
    if (c->ls_merit) {
        const double eps = 2.220446049250313e-16;
        const double m0 = c->phi0 + c->nu * c->theta, dm = c->dphi - c->nu * c->theta;
        const double mt = pht + c->nu * tht;
        c->merit_trials += 1;
        if (T[5] == 0.0 && isfinite(mt) && mt <= m0 + o.armijo * alpha * dm + 10.0 * eps * fabs(m0)) {
            c->filter_n = 0;
            c->phase = kPhU;
            return;
        }
        c->alpha = 0.5 * alpha;
        if (c->merit_trials >= o.ls_max) {
            c->status = NMPC_LINESEARCH_FAIL;
            c->phase = kPhDone;
        }
        return;
    }
    if (filter_accepts(I, c, o, tht, pht, T[5] == 0.0, alpha)) {
        c->phase = kPhU;
        return;
    }
    if (c->trials == 1 && T[5] == 0.0 && isfinite(tht) && tht >= c->theta && o.soc_max > 0) {
        c->alpha0 = alpha;
        c->soc_p = 0;
        c->soc_theta = c->theta;
        c->phase = kPhC;
        return;
    }
    const double next = 0.5 * alpha;
    c->alpha = next;
    if (next < c->amin || c->trials >= o.ls_max) filter_search_failed(c, o);
}

// ---- second-order corrections --------------------------------------------------------
// Corrected residual per lifted row, r4s = a r4s + (g^l + s) at the last trial
// point (first correction: a = alpha0, r4s = r4), and its row combinations as
// in the assembly.
__global__ void __launch_bounds__(kBlock) k_soc_rows(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const Ctl* c = I.ctl;
    if (!ctl_active(c, kPhC)) return;
    const int r = lb * kBlock + threadIdx.x;
    if (r >= I.m) return;
    const bool first = c->soc_p == 0;
    const double a = first ? c->alpha0 : c->soc_a;
    const double gamma = c->gamma;
    const double* prev = first ? I.r4 : I.r4s;
    auto corr = [&](int l) { return a * prev[l] + (lifted_g(I, gamma, l) + I.st[l]); };
    if (r < I.mc) {
        const int la = r, lbr = I.mc + r;
        const double ra = corr(la), rb = corr(lbr);
        I.r4s[la] = ra;
        I.r4s[lbr] = rb;
        I.vcomb_s[r] = (I.Q[la] * ra - I.r2[la]) - (I.Q[lbr] * rb - I.r2[lbr]);
    } else {
        const int la = I.mc + r;
        const double ra = corr(la);
        I.r4s[la] = ra;
        I.vcomb_s[r] = I.Q[la] * ra - I.r2[la];
    }
}

// rhs_s = -r1 - G^T (Q r4s - r2)
__global__ void __launch_bounds__(kBlock) k_soc_vars(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    if (!ctl_active(I.ctl, kPhC)) return;
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n) return;
    const double acc = gather_sum(
        I.jt_ptr[j], I.jt_ptr[j + 1], 0.0, [&](int e) { return int2{I.jt_row[e], I.jt_slot[e]}; },
        [&](int2 rs) { return I.jv[rs.y] * I.vcomb_s[rs.x]; });
    I.rhs_s[j] = -I.r1v[j] - acc;
}

// directions of the correction and their fraction-to-boundary bounds
// q: 0 alpha_primal(min) 1 alpha_dual(min)
constexpr Ops kOpsC{2, {kMin, kMin}};
__global__ void __launch_bounds__(kBlock) k_soc_dirs(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, kPhC)) return;
    const double mu = I.ctl->mu, tau = I.ctl->tau;
    double q[2] = {INFINITY, INFINITY};
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.m) {
        const int r = t;
        double jdy = 0.0;
        for (int p = I.jptr[r]; p < I.jptr[r + 1]; ++p) jdy += I.jv[p] * I.dy_s[I.jcol[p]];
        const int nl = r < I.mc ? 2 : 1;
        for (int h = 0; h < nl; ++h) {
            const int l = r < I.mc ? (h == 0 ? r : I.mc + r) : I.mc + r;
            const double sgn = (r < I.mc && h == 1) ? -1.0 : 1.0;
            const double sl = I.s[l], Ql = I.Q[l];
            const double dsl = -I.r4s[l] - sgn * jdy;
            const double dbel = mu / sl - I.be[l] - Ql * dsl;
            I.ds_s[l] = dsl;
            I.dom_s[l] = -I.r2[l] - Ql * dsl;
            I.dbe_s[l] = dbel;
            q[0] = fmin(q[0], ftb(sl, dsl, tau));
            q[1] = fmin(q[1], ftb(I.be[l], dbel, tau));
        }
    } else if (t < I.m + I.n) {
        const int j = t - I.m;
        const bool hl = hasL(I, j), hu = hasU(I, j);
        const double gl = hl ? I.y[j] - I.lb[j] : 1.0;
        const double gu = hu ? I.ub[j] - I.y[j] : 1.0;
        const double dyj = I.dy_s[j];
        const double zl = hl ? I.zl[j] : 0.0, zu = hu ? I.zu[j] : 0.0;
        const double dzlj = hl ? mu / gl - zl - (zl / gl) * dyj : 0.0;
        const double dzuj = hu ? mu / gu - zu + (zu / gu) * dyj : 0.0;
        I.dzl_s[j] = dzlj;
        I.dzu_s[j] = dzuj;
        if (hl) {
            q[0] = fmin(q[0], ftb(gl, dyj, tau));
            q[1] = fmin(q[1], ftb(zl, dzlj, tau));
        }
        if (hu) {
            q[0] = fmin(q[0], ftb(gu, -dyj, tau));
            q[1] = fmin(q[1], ftb(zu, dzuj, tau));
        }
    }
    store_partials(q, kOpsC, I.part, nblocks_of(sp, inst), lb, sh);
}

__global__ void __launch_bounds__(kBlock) k_soc_bound(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double E[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (c->phase != kPhC) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsC, sh, E);
    if (threadIdx.x == 0) c->soc_a = fmin(fmin(1.0, E[0]), fmin(1.0, E[1]));
}

__global__ void __launch_bounds__(kBlock) k_soc_point(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    if (!ctl_active(I.ctl, kPhC)) return;
    const double a = I.ctl->soc_a;
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) I.yt[t] = I.y[t] + a * I.dy_s[t];
    if (t < I.ml) I.st[t] = I.s[t] + a * I.ds_s[t];
}

// Verdict on the corrected trial point: accept (the update takes the
// correction's direction and step), try another correction, or fall back to
// halving the first trial step.
__global__ void __launch_bounds__(kBlock) k_decideC(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double T[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (c->phase != kPhC) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsT, sh, T);
    if (threadIdx.x != 0) return;
    const double mu = c->mu;
    const double pht = T[0] - mu * T[1] - mu * T[2] - mu * T[3];
    const double tht = T[4];
    const bool finite = T[5] == 0.0;
    if (filter_accepts(I, c, o, tht, pht, finite, c->alpha0)) {
        c->use_soc = 1;
        c->alpha = c->soc_a;
        c->phase = kPhU;
        return;
    }
    if (finite && isfinite(tht) && tht <= o.soc_kappa * c->soc_theta && c->soc_p + 1 < o.soc_max) {
        c->soc_p += 1;
        c->soc_theta = tht;
        return;
    }
    const double next = 0.5 * c->alpha0;
    c->alpha = next;
    if (next < c->amin || c->trials >= o.ls_max) {
        filter_search_failed(c, o);
    } else {
        c->phase = kPhT;
    }
}

// z <- z + alpha dz, then keep beta, zL, zU within kappa_sigma of mu / (slack or gap)
__global__ void __launch_bounds__(kBlock) k_update(const InstPtrs* __restrict__ Ia, Space sp, double ks) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!ctl_active(I.ctl, kPhU)) return;
    const double alpha = I.ctl->alpha, mu = I.ctl->mu;
    const bool soc = I.ctl->use_soc != 0;
    const double* __restrict__ dy = soc ? I.dy_s : I.dy;
    const double* __restrict__ ds = soc ? I.ds_s : I.ds;
    const double* __restrict__ dom = soc ? I.dom_s : I.dom;
    const double* __restrict__ dbe = soc ? I.dbe_s : I.dbe;
    const double* __restrict__ dzl = soc ? I.dzl_s : I.dzl;
    const double* __restrict__ dzu = soc ? I.dzu_s : I.dzu;
    const int t = lb * kBlock + threadIdx.x;
    // every load of the thread's variable and lifted row is issued before the
    // first store
    const bool var = t < I.n, hyk = I.ctl->hyk != 0;
    const bool row = t < I.ml && !(hyk && t < 2 * I.mc), lam = hyk && t < I.mc;
    double yj = 0.0, dyj = 0.0, lbj = 0.0, ubj = 0.0, zlj = 0.0, zuj = 0.0, dzlj = 0.0, dzuj = 0.0;
    if (var) {
        yj = I.y[t]; dyj = dy[t]; lbj = I.lb[t]; ubj = I.ub[t];
        zlj = I.zl[t]; zuj = I.zu[t]; dzlj = dzl[t]; dzuj = dzu[t];
    }
    double sr = 0.0, dsr = 0.0, omr = 0.0, domr = 0.0, ber = 0.0, dber = 0.0;
    if (row) {
        sr = I.s[t]; dsr = ds[t]; ber = I.be[t]; dber = dbe[t];
    }
    if (row || lam) {
        omr = I.om[t]; domr = dom[t];
    }
    if (var) {
        const int j = t;
        const double yn = yj + alpha * dyj;
        I.y[j] = yn;
        if (lbj > -INFINITY) {
            const double gl = yn - lbj;
            const double z = zlj + alpha * dzlj;
            I.zl[j] = fmin(fmax(z, mu / (ks * gl)), ks * mu / gl);
        } else {
            I.zl[j] = 0.0;
        }
        if (ubj < INFINITY) {
            const double gu = ubj - yn;
            const double z = zuj + alpha * dzuj;
            I.zu[j] = fmin(fmax(z, mu / (ks * gu)), ks * mu / gu);
        } else {
            I.zu[j] = 0.0;
        }
    }
    if (lam) {
        I.om[t] = omr + alpha * domr;   // HyKKT: lambda; no slack or slack dual
    } else if (row) {
        const int r = t;
        const double sn = sr + alpha * dsr;
        I.s[r] = sn;
        I.om[r] = omr + alpha * domr;
        const double b = ber + alpha * dber;
        I.be[r] = fmin(fmax(b, mu / (ks * sn)), ks * mu / sn);
    }
}

// End of a pass: accepted instances start their next iteration; count the
// instances still running.
__global__ void __launch_bounds__(kBlock) k_pass_end(const InstPtrs* __restrict__ Ia, int ninst, int* running) {
    __shared__ int cnt, csoc;
    if (threadIdx.x == 0) cnt = csoc = 0;
    __syncthreads();
    int mine = 0, soc = 0;
    for (int i = threadIdx.x; i < ninst; i += kBlock) {
        Ctl* c = Ia[i].ctl;
        if (c->phase == kPhU) {
            c->it += 1;
            c->phase = kPhA;
        }
        if (c->phase != kPhDone) ++mine;
        if (c->phase == kPhC) ++soc;
    }
    if (mine) atomicAdd(&cnt, mine);
    if (soc) atomicAdd(&csoc, soc);
    __syncthreads();
    if (threadIdx.x == 0) {
        running[0] = cnt;
        running[1] = csoc;
    }
}

// cold start: push y into the bounds' interior (bound_push of magnitude and range)
__global__ void __launch_bounds__(kBlock) k_push_bounds(const InstPtrs* __restrict__ Ia, Space sp, double bp) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n) return;
    const bool hl = hasL(I, j), hu = hasU(I, j);
    double pl = hl ? bp * fmax(1.0, fabs(I.lb[j])) : 0.0;
    double pu = hu ? bp * fmax(1.0, fabs(I.ub[j])) : 0.0;
    if (hl && hu) {
        const double rng = I.ub[j] - I.lb[j];
        pl = fmin(pl, 0.5 * bp * rng);
        pu = fmin(pu, 0.5 * bp * rng);
    }
    double v = I.y[j];
    if (hl) v = fmax(v, I.lb[j] + pl);
    if (hu) v = fmin(v, I.ub[j] - pu);
    I.y[j] = v;
}

// cold start: slacks, multipliers centred at mu0
__global__ void __launch_bounds__(kBlock)
k_cold_duals(const InstPtrs* __restrict__ Ia, Space sp, double mu0, double spush) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    const double gamma = I.ctl->gamma;
    const int t = lb * kBlock + threadIdx.x;
    if (t < 2 * I.mc && I.ctl->hyk) {   // HyKKT: lambda = 0; the slack slots of equality rows stay inert
        I.s[t] = 1.0;
        I.om[t] = 0.0;
        I.be[t] = 0.0;
    } else if (t < I.ml) {
        const double g = lifted_g(I, gamma, t);
        const double sv = fmax(-g, spush * fmax(1.0, fabs(g)));
        I.s[t] = sv;
        I.om[t] = 0.0;
        I.be[t] = mu0 / sv;
    }
    if (t < I.n) {
        I.zl[t] = hasL(I, t) ? mu0 / (I.y[t] - I.lb[t]) : 0.0;
        I.zu[t] = hasU(I, t) ? mu0 / (I.ub[t] - I.y[t]) : 0.0;
    }
}

__global__ void k_set_fail(const InstPtrs* __restrict__ Ia, int ninst, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ninst) Ia[i].ctl->fail = value;
}

// ---- sensitivities ------------------------------------------------------------------
// rhs = seed_obj * grad f + S_u^T seed_u (first-stage controls at positions nx .. nx + nu);
// the seed sits in adj_seed (u part, then seed_obj)
__global__ void __launch_bounds__(kBlock) k_adj_seed(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n) return;
    double v = I.adj_seed[I.nu] * I.grad[j];
    if (j >= I.nx && j < I.nx + I.nu) v += I.adj_seed[j - I.nx];
    I.adj_b[j] = v;
    I.adj_rhs[j] = v;
}

// cold start, first guess: every stage holds the measured state and the last
// control (the reflux column also its equilibrium vapour and the flows)
__global__ void __launch_bounds__(kBlock) k_cold_guess(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n || I.family == NMPC_FAMILY_STAGE_MODEL) return;   // stage models: their own guess kernel
    const int r = j % I.ns;
    double v;
    if (r < I.nx) {
        v = I.x0[r];
    } else if (r < I.nx + I.nu) {
        v = I.uprev[r - I.nx];
    } else {   // reflux column: y_i = phi(x0_i), then L = u D, V = L + D, S = L + F
        const RefluxConst& C = I.rc;
        const int N = I.rd.N;
        if (r <= 2 * N) {
            const double x = I.x0[r - N - 1];
            v = C.alpha * x / (1.0 + (C.alpha - 1.0) * x);
        } else {
            const double L = I.uprev[0] * C.D;
            v = r == 2 * N + 1 ? L : (r == 2 * N + 2 ? L + C.D : L + C.F);
        }
    }
    I.y[j] = v;
}

__device__ inline double row_dot(const InstPtrs& I, int r, const double* __restrict__ v) {
    double acc = 0.0;
    for (int p = I.jptr[r]; p < I.jptr[r + 1]; ++p) acc += I.jv[p] * v[I.jcol[p]];
    return acc;
}

// lam = Q (J w) per original row (Q = qeff: Q+ + Q- on c rows, Q_d on d rows)
__global__ void __launch_bounds__(kBlock) k_adj_lam(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int r = lb * kBlock + threadIdx.x;
    if (r >= I.m) return;
    I.adj_lam[r] = I.qeff[r] * row_dot(I, r, I.adj_w);
}

// qr = Q (Q^{-1} lam - J w) = lam - Q (J w)
__global__ void __launch_bounds__(kBlock) k_adj_qr(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int r = lb * kBlock + threadIdx.x;
    if (r >= I.m) return;
    I.adj_qr[r] = I.adj_lam[r] - I.qeff[r] * row_dot(I, r, I.adj_w);
}

// adj_rhs = b - (W + Sigma + eta I) w - J^T lam + J^T qr
__global__ void __launch_bounds__(kBlock) k_adj_rho(const InstPtrs* __restrict__ Ia, Space sp, double eta) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int j = lb * kBlock + threadIdx.x;
    if (j >= I.n) return;
    const double* w = I.adj_w;
    double acc = I.adj_b[j] - (I.sig[j] + eta) * w[j];
    for (int e = I.wf_ptr[j]; e < I.wf_ptr[j + 1]; ++e) acc -= I.wv[I.wf_slot[e]] * w[I.wf_col[e]];
    for (int e = I.jt_ptr[j]; e < I.jt_ptr[j + 1]; ++e) {
        const int r = I.jt_row[e];
        acc += I.jv[I.jt_slot[e]] * (I.adj_qr[r] - I.adj_lam[r]);
    }
    I.adj_rhs[j] = acc;
}

// w += d; lam += Q (J d) - qr
__global__ void __launch_bounds__(kBlock) k_adj_update(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.m) I.adj_lam[t] += I.qeff[t] * row_dot(I, t, I.adj_d) - I.adj_qr[t];
    if (t < I.n) I.adj_w[t] += I.adj_d[t];
}

// Parameter contractions of w = K^{-1} seed for the distillation family (one block),
// with lam = (Q+ + Q-) (J w) the refined multiplier of the uncondensed solve
// (recomputing Q (J w) from w would multiply the rounding of J w by Q):
//   x0:       lam on the stage-1 rows
//   zF_k:     dt F lam on the feed-tray row of stage k
//   xD*, xB*: 2 sum_k w(top|bottom state) - 2 seed_obj sum_k (state - setpoint)
//   u_prev:   2 rho w(u_1) - 2 rho seed_obj (u_1 - u_prev)
// out = [x0 (nx) | setpoint (2) | traj (H) | u_prev (2)]
__global__ void __launch_bounds__(kBlock) k_adj_gather_distill(const InstPtrs* __restrict__ Ia) {
    __shared__ double sh[kMaxQ * kWaves];
    const InstPtrs& I = Ia[0];
    const double seed_obj = I.adj_seed[I.nu];
    const DistillDims D = I.dd;
    const DistillConst C = I.dc;
    const double* w = I.adj_w;
    const double* y = I.y;
    double* out = I.adj_out;
    const int tid = threadIdx.x;
    for (int t = tid; t < D.nx + D.H; t += kBlock) {
        const int r = t < D.nx ? t : (t - D.nx) * D.nx + D.fd;
        const double v = I.adj_lam[r];
        if (t < D.nx) out[t] = v;
        else out[D.nx + 2 + (t - D.nx)] = C.dt * C.F * v;
    }
    const double xD = I.setp[0], xB = I.setp[1];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < D.H; k += kBlock) {
        const int top = k * D.ns, bot = k * D.ns + D.nx - 1;
        a[0] += w[top];
        a[1] += y[top] - xD;
        a[2] += w[bot];
        a[3] += y[bot] - xB;
    }
    constexpr Ops ops{4, {kSum, kSum, kSum, kSum}};
    const double r = block_reduce(a, ops, sh);
    __shared__ double tot[4];
    if (tid < 4) tot[tid] = r;
    __syncthreads();
    if (tid == 0) {
        out[D.nx] = 2.0 * tot[0] - 2.0 * seed_obj * tot[1];
        out[D.nx + 1] = 2.0 * tot[2] - 2.0 * seed_obj * tot[3];
    }
    if (tid < 2) {
        const int iu = D.nx + tid;
        out[D.nx + 2 + D.H + tid] = 2.0 * C.rho * w[iu] - 2.0 * C.rho * seed_obj * (y[iu] - I.uprev[tid]);
    }
}

// Parameter contractions of w = K^{-1} seed for the plate family:
//   x0_p:  lam = (Q+ + Q-) (J w), the refined multiplier, on the stage-1 row of node p
//   T*_p:  2 sum_k w(T_kp) - 2 seed_obj sum_k (T_kp - T*_p)
//   u_prev: 0 (it enters no function of the problem)
// out = [x0 (nx) | setpoint (nx) | u_prev (16)]; one thread per node.
__global__ void __launch_bounds__(kBlock) k_adj_gather_plate(const InstPtrs* __restrict__ Ia) {
    const InstPtrs& I = Ia[0];
    const double seed_obj = I.adj_seed[I.nu];
    const PlateDims D = I.pd;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    double* out = I.adj_out;
    if (p < I.nu) out[2 * D.nx + p] = 0.0;
    if (p >= D.nx) return;
    out[p] = I.adj_lam[p];
    double sw = 0.0, sd = 0.0;
    const double tgt = I.setp[p];
    for (int k = 0; k < D.H; ++k) {
        sw += I.adj_w[(int64_t)k * D.ns + p];
        sd += I.y[(int64_t)k * D.ns + p] - tgt;
    }
    out[D.nx + p] = 2.0 * sw - 2.0 * seed_obj * sd;
}

// Parameter contractions for the reflux column (one block): the objective is
// dt sum_k (x_{k,1} - xbar)^2 + w_u (u_k - ubar)^2, so
//   x0:     lam on the stage-1 tray rows
//   xbar:   2 dt sum_k w(x_{k,1}) - 2 dt seed_obj sum_k (x_{k,1} - xbar)
//   ubar:   2 dt w_u sum_k w(u_k) - 2 dt w_u seed_obj sum_k (u_k - ubar)
//   u_prev: 0 (it enters no function of the problem)
// out = [x0 (N) | setpoint (2) | u_prev (1)]
__global__ void __launch_bounds__(kBlock) k_adj_gather_reflux(const InstPtrs* __restrict__ Ia) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double tot[4];
    const InstPtrs& I = Ia[0];
    const RefluxDims D = I.rd;
    const RefluxConst C = I.rc;
    const double seed_obj = I.adj_seed[I.nu];
    const double xbar = I.setp[0], ubar = I.setp[1];
    double* out = I.adj_out;
    const int tid = threadIdx.x;
    for (int t = tid; t < D.N; t += kBlock) out[t] = I.adj_lam[t];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = tid; k < D.H; k += kBlock) {
        const int64_t o = (int64_t)k * D.ns;
        a[0] += I.adj_w[o];
        a[1] += I.y[o] - xbar;
        a[2] += I.adj_w[o + D.N];
        a[3] += I.y[o + D.N] - ubar;
    }
    constexpr Ops ops{4, {kSum, kSum, kSum, kSum}};
    const double r = block_reduce(a, ops, sh);
    if (tid < 4) tot[tid] = r;
    __syncthreads();
    if (tid == 0) {
        out[D.N] = 2.0 * C.dt * tot[0] - 2.0 * C.dt * seed_obj * tot[1];
        out[D.N + 1] = 2.0 * C.dt * C.wu * tot[2] - 2.0 * C.dt * C.wu * seed_obj * tot[3];
        out[D.N + 2] = 0.0;
    }
}

// ---- shifted warm start -----------------------------------------------------------------
// Stage k takes stage k + 1's values, the last stage keeps its own: variables by
// stages of ns; lifted rows [plus | minus | inequality] with the stage-major
// equality rows by stages of rps, the hold rows of the control horizon by held
// stages of two, the inequality rows by stages of md / H.
__device__ inline int shift_src_var(const InstPtrs& I, int j) {
    const int k = j / I.ns;
    return k < I.H - 1 ? j + I.ns : j;
}

__device__ inline int shift_src_row(const InstPtrs& I, int l) {
    if (l >= 2 * I.mc) {   // I.md > 0 here: the inequality rows, md / H per stage
        const int nd = I.md / I.H;
        const int k = (l - 2 * I.mc) / nd;
        return k < I.H - 1 ? l + nd : l;
    }
    const int r = l >= I.mc ? l - I.mc : l;
    const int dyn = I.H * I.rps;
    if (r < dyn) return r / I.rps < I.H - 1 ? l + I.rps : l;
    const int hc = I.family == NMPC_FAMILY_DISTILLATION ? I.dd.hc : I.H;
    return hc + (r - dyn) / 2 < I.H - 1 ? l + 2 : l;
}

// gather the shifted iterate into the trial / direction buffers ...
__global__ void __launch_bounds__(kBlock) k_shift_gather(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) {
        const int j = shift_src_var(I, t);
        I.yt[t] = I.y[j];
        I.dzl[t] = I.zl[j];
        I.dzu[t] = I.zu[j];
    }
    if (t < I.ml) {
        const int l = shift_src_row(I, t);
        I.st[t] = I.s[l];
        I.dom[t] = I.om[l];
        I.dbe[t] = I.be[l];
    }
}

// ... and take it as the iterate
__global__ void __launch_bounds__(kBlock) k_shift_take(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int t = lb * kBlock + threadIdx.x;
    if (t < I.n) {
        I.y[t] = I.yt[t];
        I.zl[t] = I.dzl[t];
        I.zu[t] = I.dzu[t];
    }
    if (t < I.ml) {
        I.s[t] = I.st[t];
        I.om[t] = I.dom[t];
        I.be[t] = I.dbe[t];
    }
}

// ---- HyKKT: conjugate gradients on S = J_c K_gamma^{-1} J_c^T --------------------------
// After the solve K_gamma w0 = b1 + gamma_h J_c^T b2 (w0 in dy), S x = J_c w0 - b2
// (b2 = -c) is solved by CG from x = 0; every product with S is J_c^T p, one
// solve with the factor (hk_t -> hk_w), then J_c w.  Equality rows only.
constexpr Ops kOpsSum1{1, {kSum}};

__device__ inline bool hk_step(const Ctl* c) { return c->phase == kPhS && c->hyk; }
__device__ inline bool hk_cg_running(const Ctl* c) { return hk_step(c) && !c->cg_done; }

// J_c^T v over the equality rows, for variable j
__device__ inline double hk_jct(const InstPtrs& I, int j, const double* __restrict__ v) {
    return gather_sum(
        I.jt_ptr[j], I.jt_ptr[j + 1], 0.0, [&](int e) { return int2{I.jt_row[e], I.jt_slot[e]}; },
        [&](int2 rs) { return rs.x < I.mc ? I.jv[rs.y] * v[rs.x] : 0.0; });
}

// r = p = J_c w0 + c, x = 0; partial |r|^2
__global__ void __launch_bounds__(kBlock) k_hk_cg_init(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!hk_step(I.ctl)) return;
    double q[1] = {0.0};
    const int r = lb * kBlock + threadIdx.x;
    if (r < I.mc) {
        const double b = row_dot(I, r, I.dy) + I.c[r];
        I.hk_r[r] = b;
        I.hk_p[r] = b;
        I.hk_x[r] = 0.0;
        q[0] = b * b;
    }
    store_partials(q, kOpsSum1, I.part, nblocks_of(sp, inst), lb, sh);
}

__global__ void __launch_bounds__(kBlock) k_hk_cg_begin(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double T[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (!hk_step(c)) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsSum1, sh, T);
    if (threadIdx.x != 0) return;
    c->cg_rr = T[0];
    c->cg_stop = o.cg_tol * sqrt(T[0]);
    c->cg_it = 0;
    c->cg_done = (T[0] == 0.0 || o.cg_max <= 0) ? 1 : 0;
}

// hk_t = J_c^T p
__global__ void __launch_bounds__(kBlock) k_hk_jt(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    if (!hk_cg_running(I.ctl)) return;
    const int j = lb * kBlock + threadIdx.x;
    if (j < I.n) I.hk_t[j] = hk_jct(I, j, I.hk_p);
}

// Sp = J_c hk_w; partial p . Sp
__global__ void __launch_bounds__(kBlock) k_hk_sp(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!hk_cg_running(I.ctl)) return;
    double q[1] = {0.0};
    const int r = lb * kBlock + threadIdx.x;
    if (r < I.mc) {
        const double v = row_dot(I, r, I.hk_w);
        I.hk_sp[r] = v;
        q[0] = I.hk_p[r] * v;
    }
    store_partials(q, kOpsSum1, I.part, nblocks_of(sp, inst), lb, sh);
}

__global__ void __launch_bounds__(kBlock) k_hk_cg_alpha(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double T[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (!hk_cg_running(c)) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsSum1, sh, T);
    if (threadIdx.x == 0) c->cg_alpha = c->cg_rr / T[0];
}

// x += alpha p, r -= alpha Sp; partial |r|^2
__global__ void __launch_bounds__(kBlock) k_hk_axpy(const InstPtrs* __restrict__ Ia, Space sp) {
    __shared__ double sh[kMaxQ * kWaves];
    int lb;
    const int inst = block_inst(sp, lb);
    const InstPtrs& I = Ia[inst];
    if (!hk_cg_running(I.ctl)) return;
    const double a = I.ctl->cg_alpha;
    double q[1] = {0.0};
    const int r = lb * kBlock + threadIdx.x;
    if (r < I.mc) {
        I.hk_x[r] += a * I.hk_p[r];
        const double v = I.hk_r[r] - a * I.hk_sp[r];
        I.hk_r[r] = v;
        q[0] = v * v;
    }
    store_partials(q, kOpsSum1, I.part, nblocks_of(sp, inst), lb, sh);
}

// convergence (|r| <= cg_tol |b|) or the iteration limit; otherwise beta
__global__ void __launch_bounds__(kBlock) k_hk_cg_beta(const InstPtrs* __restrict__ Ia, Space sp, DevOpts o) {
    __shared__ double sh[kMaxQ * kWaves];
    __shared__ double T[kMaxQ];
    const int inst = blockIdx.x;
    const InstPtrs& I = Ia[inst];
    Ctl* c = I.ctl;
    if (!hk_cg_running(c)) return;
    finalize_partials(I.part, nblocks_of(sp, inst), kOpsSum1, sh, T);
    if (threadIdx.x != 0) return;
    const double rr = T[0];
    c->cg_it += 1;
    c->cg_total += 1;
    if (sqrt(rr) <= c->cg_stop || c->cg_it >= o.cg_max) {
        c->cg_done = 1;
    } else {
        c->cg_beta = rr / c->cg_rr;
        c->cg_rr = rr;
    }
}

// p = r + beta p
__global__ void __launch_bounds__(kBlock) k_hk_pupd(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    if (!hk_cg_running(I.ctl)) return;
    const int r = lb * kBlock + threadIdx.x;
    if (r < I.mc) I.hk_p[r] = I.hk_r[r] + I.ctl->cg_beta * I.hk_p[r];
}

// instances whose CG still runs -> *count
__global__ void __launch_bounds__(kBlock) k_hk_count(const InstPtrs* __restrict__ Ia, int ninst, int* count) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int i = threadIdx.x; i < ninst; i += kBlock) mine += hk_cg_running(Ia[i].ctl) ? 1 : 0;
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) *count = cnt;
}

// right-hand side of the final solve: b1 + gamma_h J_c^T b2 - J_c^T x
__global__ void __launch_bounds__(kBlock) k_hk_finish(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    if (!hk_step(I.ctl)) return;
    const int j = lb * kBlock + threadIdx.x;
    if (j < I.n) I.rhs[j] -= hk_jct(I, j, I.hk_x);
}

// a Lifted-KKT iterate as a HyKKT one: lambda = omega+ - omega-, the equality
// rows' slack slots inert
__global__ void __launch_bounds__(kBlock) k_hk_from_lifted(const InstPtrs* __restrict__ Ia, Space sp) {
    int lb;
    const InstPtrs& I = Ia[block_inst(sp, lb)];
    const int r = lb * kBlock + threadIdx.x;
    if (r >= I.mc) return;
    const int b = I.mc + r;
    I.om[r] = I.om[r] - I.om[b];
    I.om[b] = 0.0;
    I.s[r] = 1.0;
    I.s[b] = 1.0;
    I.be[r] = 0.0;
    I.be[b] = 0.0;
}

}  // namespace

void launch_phaseA(const InstPtrs* I, const IpmSpaces& S, int ninst, int pred, const DevOpts& o, bool decide,
                   hipStream_t st) {
    const Space& sp = S.sp[kSpNML];
    hipLaunchKernelGGL(k_phaseA, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, pred);
    if (decide) hipLaunchKernelGGL(k_decideA, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
}

void launch_assemble(const InstPtrs* I, const IpmSpaces& S, int pred, hipStream_t st) {
    hipLaunchKernelGGL(k_rows_prep, dim3(S.sp[kSpM].blocks), dim3(kBlock), 0, st, I, S.sp[kSpM], pred);
    hipLaunchKernelGGL(k_var_prep, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN], pred);
    hipLaunchKernelGGL(k_assemble, dim3(S.sp[kSpK].blocks), dim3(kBlock), 0, st, I, S.sp[kSpK], pred);
}

void launch_decideF(const InstPtrs* I, int ninst, const DevOpts& o, hipStream_t st) {
    hipLaunchKernelGGL(k_decideF, dim3((ninst + 63) / 64), dim3(64), 0, st, I, ninst, o);
}

void launch_phaseE(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st) {
    const Space& sp = S.sp[kSpMN];
    hipLaunchKernelGGL(k_phaseE, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_decideE, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
}

void launch_trial(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    hipLaunchKernelGGL(k_trial_point, dim3(S.sp[kSpMax].blocks), dim3(kBlock), 0, st, I, S.sp[kSpMax]);
}

void launch_phaseT(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st) {
    const Space& sp = S.sp[kSpNML];
    hipLaunchKernelGGL(k_phaseT, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, (int)kPhT);
    hipLaunchKernelGGL(k_decideT, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
}

void launch_soc_prepare(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    hipLaunchKernelGGL(k_soc_rows, dim3(S.sp[kSpM].blocks), dim3(kBlock), 0, st, I, S.sp[kSpM]);
    hipLaunchKernelGGL(k_soc_vars, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN]);
}

void launch_soc_step(const InstPtrs* I, const IpmSpaces& S, int ninst, hipStream_t st) {
    const Space& sp = S.sp[kSpMN];
    hipLaunchKernelGGL(k_soc_dirs, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_soc_bound, dim3(ninst), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_soc_point, dim3(S.sp[kSpMax].blocks), dim3(kBlock), 0, st, I, S.sp[kSpMax]);
}

void launch_soc_decide(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st) {
    const Space& sp = S.sp[kSpNML];
    hipLaunchKernelGGL(k_phaseT, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp, (int)kPhC);
    hipLaunchKernelGGL(k_decideC, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
}

void launch_update(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* running,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(S.sp[kSpMax].blocks), dim3(kBlock), 0, st, I, S.sp[kSpMax], o.kappa_sigma);
    hipLaunchKernelGGL(k_pass_end, dim3(1), dim3(kBlock), 0, st, I, ninst, running);
}

void launch_cold_start(const InstPtrs* I, const IpmSpaces& S, double bound_push, double slack_push, double mu0,
                       bool after_eval, hipStream_t st) {
    if (!after_eval)
        hipLaunchKernelGGL(k_push_bounds, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN], bound_push);
    else
        hipLaunchKernelGGL(k_cold_duals, dim3(S.sp[kSpMax].blocks), dim3(kBlock), 0, st, I, S.sp[kSpMax], mu0,
                           slack_push);
}

void launch_set_fail(const InstPtrs* I, int ninst, int value, hipStream_t st) {
    hipLaunchKernelGGL(k_set_fail, dim3((ninst + 63) / 64), dim3(64), 0, st, I, ninst, value);
}

void launch_adj_seed(const InstPtrs* I, const Space& spN, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_seed, dim3(spN.blocks), dim3(kBlock), 0, st, I, spN);
}

// lam = omega+ - omega- (equality multipliers of the original problem) and the
// multipliers of the inequality rows, written to caller buffers (instance 0)
__global__ void __launch_bounds__(kBlock) k_export_duals(const InstPtrs* __restrict__ Ia, double* lam, double* om_d) {
    const InstPtrs& I = Ia[0];
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (lam && r < I.mc) lam[r] = I.om[r] - I.om[I.mc + r];
    if (om_d && r < I.md) om_d[r] = I.om[2 * I.mc + r];
}

void launch_export_duals(const InstPtrs* I, double* lam, double* om_d, int rows, hipStream_t st) {
    if (rows > 0) hipLaunchKernelGGL(k_export_duals, dim3((rows + kBlock - 1) / kBlock), dim3(kBlock), 0, st, I, lam, om_d);
}

void launch_cold_guess(const InstPtrs* I, const Space& spN, hipStream_t st) {
    hipLaunchKernelGGL(k_cold_guess, dim3(spN.blocks), dim3(kBlock), 0, st, I, spN);
}

void launch_adj_refine(int step, const InstPtrs* I, const IpmSpaces& S, double eta, hipStream_t st) {
    const Space& spM = S.sp[kSpM];
    if (step == 0) {
        hipLaunchKernelGGL(k_adj_lam, dim3(spM.blocks), dim3(kBlock), 0, st, I, spM);
    } else if (step == 1) {
        hipLaunchKernelGGL(k_adj_qr, dim3(spM.blocks), dim3(kBlock), 0, st, I, spM);
        hipLaunchKernelGGL(k_adj_rho, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN], eta);
    } else {
        hipLaunchKernelGGL(k_adj_update, dim3(S.sp[kSpMax].blocks), dim3(kBlock), 0, st, I, S.sp[kSpMax]);
    }
}

void launch_hk_cg_start(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* count,
                        hipStream_t st) {
    const Space& sp = S.sp[kSpM];
    hipLaunchKernelGGL(k_hk_cg_init, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_hk_cg_begin, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
    hipLaunchKernelGGL(k_hk_count, dim3(1), dim3(kBlock), 0, st, I, ninst, count);
}

void launch_hk_cg_pre(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    hipLaunchKernelGGL(k_hk_jt, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN]);
}

void launch_hk_cg_post(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* count,
                       hipStream_t st) {
    const Space& sp = S.sp[kSpM];
    hipLaunchKernelGGL(k_hk_sp, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_hk_cg_alpha, dim3(ninst), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_hk_axpy, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_hk_cg_beta, dim3(ninst), dim3(kBlock), 0, st, I, sp, o);
    hipLaunchKernelGGL(k_hk_pupd, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_hk_count, dim3(1), dim3(kBlock), 0, st, I, ninst, count);
}

void launch_hk_finish(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    hipLaunchKernelGGL(k_hk_finish, dim3(S.sp[kSpN].blocks), dim3(kBlock), 0, st, I, S.sp[kSpN]);
}

void launch_shift(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    const Space& sp = S.sp[kSpMax];
    hipLaunchKernelGGL(k_shift_gather, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
    hipLaunchKernelGGL(k_shift_take, dim3(sp.blocks), dim3(kBlock), 0, st, I, sp);
}

void launch_hk_from_lifted(const InstPtrs* I, const IpmSpaces& S, hipStream_t st) {
    hipLaunchKernelGGL(k_hk_from_lifted, dim3(S.sp[kSpM].blocks), dim3(kBlock), 0, st, I, S.sp[kSpM]);
}

// d u1 / d x0 of a stage model whose state rows hold the previous states
// through the matrix C (pc): row k is -C^T lam_k over the first stage's state
// rows (lam_k: the sensitivity multipliers of seed k, stride apart).
__global__ void __launch_bounds__(kBlock) k_x0_map(const double* __restrict__ lam, int64_t stride,
                                                   const double* __restrict__ pc, double* __restrict__ out, int nx,
                                                   int K) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= nx * K) return;
    const int k = t / nx, j = t - k * nx;
    const double* l = lam + (int64_t)k * stride;
    double acc = 0.0;
    for (int i = 0; i < nx; ++i) acc -= pc[(int64_t)i * nx + j] * l[i];
    out[t] = acc;
}

void launch_x0_map(const double* lam, int64_t stride, const double* pc, double* out, int nx, int K, hipStream_t st) {
    if (nx * K > 0)
        hipLaunchKernelGGL(k_x0_map, dim3((nx * K + kBlock - 1) / kBlock), dim3(kBlock), 0, st, lam, stride, pc, out,
                           nx, K);
}

void launch_adj_gather(const InstPtrs* I, int family, int nx, hipStream_t st) {
    if (family == NMPC_FAMILY_REFLUX_COLUMN)
        hipLaunchKernelGGL(k_adj_gather_reflux, dim3(1), dim3(kBlock), 0, st, I);
    else if (family == NMPC_FAMILY_HEATED_PLATE)
        hipLaunchKernelGGL(k_adj_gather_plate, dim3((nx + kBlock - 1) / kBlock), dim3(kBlock), 0, st, I);
    else
        hipLaunchKernelGGL(k_adj_gather_distill, dim3(1), dim3(kBlock), 0, st, I);
}

}  // namespace nmpc
