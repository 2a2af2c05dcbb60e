// Numeric supernodal Cholesky and triangular solves (eqs. 20-25), multifrontal
// form: supernode s owns a dense front F_s of size m_s x m_s over its row list
// R_s (its w_s own columns first).  F_s starts from the KKT entries of its
// columns, receives the update blocks of its children by extend-add through
// precomputed relative positions, and is partially factored on its first w_s
// columns; the factored columns are the L panel (eq. 21 restricted to S_L) and
// the trailing block is the update passed to the parent.
//
// Scheduling: a launch covers a list of supernode groups; workgroup b factors
// the supernodes of group b one after another.  Wide levels of the supernodal
// tree are one group per supernode (one launch per level); the narrow top of
// the tree, where each level holds one or two supernodes, is a single group
// walked by one workgroup, so a chain of fronts costs one launch.  Every sum is
// taken in a fixed order, so results do not depend on scheduling.
#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "front_chol.h"

namespace nmpc {

namespace {

constexpr int kWave = 64;

__device__ inline double shfl(double v, int lane) { return __shfl(v, lane, kWave); }

constexpr int kBatch = 8;   // independent global loads in flight per thread

// Copy n values from global to shared memory, kBatch loads in flight per thread.
template <class T>
__device__ void g2s(T* dst, const T* __restrict__ src, int64_t n) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int64_t base = 0; base < n; base += (int64_t)nthr * kBatch) {
        T v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t e = base + tid + (int64_t)u * nthr;
            v[u] = e < n ? src[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int64_t e = base + tid + (int64_t)u * nthr;
            if (e < n) dst[e] = v[u];
        }
    }
}

// Entry e of the lower triangle of an n x n matrix packed by columns, as (i, j)
// (n <= 256 here, so b^2 - 8e is exact in single precision; the integer steps
// correct the rounded root).
__device__ __attribute__((always_inline)) inline void unpack_lower(int e, int n, int& i, int& j) {
    const float b = 2.0f * (float)n + 1.0f;
    int c = (int)((b - sqrtf(b * b - 8.0f * (float)e)) * 0.5f);
    c = max(0, min(c, n - 1));
    while (c > 0 && c * n - ((c * (c - 1)) >> 1) > e) --c;
    while (c + 1 < n && (c + 1) * n - (((c + 1) * c) >> 1) <= e) ++c;
    j = c;
    i = c + (e - (c * n - ((c * (c - 1)) >> 1)));
}

// Loads of one round of a child's update block: entries e0 + tid + u nthr of
// its packed lower triangle (ne entries), each as a value and the front rows of
// its row and column (the child's relative row positions; -1: no entry).  The
// front position is formed only when the entry is added, so the round's loads
// stay in flight until then.
// A child's first round can also carry the first kUvec nthr entries of its
// update vector (fused forward solve).
constexpr int kUvec = 2;
struct ChildRound {
    double v[kBatch];
    int ri[kBatch], rj[kBatch];
    double uv[kUvec];
    int ur[kUvec];
};

__device__ __attribute__((always_inline)) inline void child_round(const double* __restrict__ Uc, const int32_t* __restrict__ rel, int nc, int ne,
                                   int e0, ChildRound& r, const double* __restrict__ uvec = nullptr) {
    const int tid = threadIdx.x, nthr = blockDim.x;
#pragma unroll
    for (int u = 0; u < kUvec; ++u) {
        const int i = tid + u * nthr;
        r.ur[u] = -1;
        r.uv[u] = 0.0;
        if (uvec && i < nc) {
            r.uv[u] = global(uvec)[i];
            r.ur[u] = global(rel)[i];
        }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
        const int e = e0 + tid + u * nthr;
        r.ri[u] = -1;
        r.rj[u] = 0;
        r.v[u] = 0.0;
        if (e < ne) {
            int i, j;
            unpack_lower(e, nc, i, j);
            r.v[u] = global(Uc)[i + (int64_t)j * nc];
            r.ri[u] = global(rel)[i];
            r.rj[u] = global(rel)[j];
        }
    }
}

// A child record read through a global-address-space pointer (field by field:
// a structure copy does not cross address spaces).
__device__ __attribute__((always_inline)) inline ChildRec child_rec_at(const ChildRec* recs, int k) {
    const auto* g = global(recs) + k;
    ChildRec r;
    r.u_off = g->u_off;
    r.rel_off = g->rel_off;
    r.uv_off = g->uv_off;
    r.nc = g->nc;
    r.child = g->child;
    return r;
}

// The group's first supernode, or -1 when the instance is not in the launch's
// phase.  Both reads are issued before either is waited for (groups are never
// empty, so the schedule entry exists whatever the phase).
__device__ __attribute__((always_inline)) inline int first_node(const InstPtrs& I, const Group& g, int pred) {
    const int32_t* sched = I.S.sched_nodes;
    const Ctl* c = I.ctl;   // every instance has its control block
    const int s0 = global(sched)[g.begin];
    const int ph = global(c)->phase;
    const bool active = pred == kPredAll || (pred == kPredFactor ? (ph == kPhB || ph == kPhF) : ph == pred);
    return active ? s0 : -1;
}

// One supernode: assemble the front, factor it, store the L panel and update.
// Shared-memory fronts are packed lower triangles; the global buffer of a
// medium front is square with an odd leading dimension.
template <bool Lds, int P>
__device__ __attribute__((always_inline)) void factor_one(int s, const SnView& S, const double* __restrict__ kv, double eta, double* __restrict__ L,
                           double* __restrict__ U, int* __restrict__ fail, double* F, double* v, const InstPtrs& I,
                           bool fwd) {
    using Idx = typename std::conditional<Lds, PackedIdx, SquareIdx>::type;
    // the first two children's records hang off the supernode itself, so they
    // are read with its sizes (one level of dependent loads less for the rounds)
    const ChildRec rec0 = child_rec_at(S.first_recs, 2 * s), rec1 = child_rec_at(S.first_recs, 2 * s + 1);
    const int f = global(S.sn_ptr)[s];
    const int w = global(S.sn_ptr)[s + 1] - f;
    const int m = (int)(global(S.rows_ptr)[s + 1] - global(S.rows_ptr)[s]);
    Idx ix;
    if constexpr (Lds) ix.m = m; else ix.ld = m | 1;
    const int nb = m - w;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave, nw = nthr / kWave;
    const bool fw = fwd && global(S.fused)[s];
    // original entries of the condensed matrix in this supernode's columns, the
    // first kBatch per thread loaded before the children's rounds (so that
    // waiting for them does not wait for the rounds); a diagonal entry's
    // position is stored complemented and takes + eta
    const int kt0 = global(S.k_ptr)[s], kt1 = global(S.k_ptr)[s + 1];
    const int c0 = global(S.child_ptr)[s], c1 = global(S.child_ptr)[s + 1];   // read with the entry range
    int kp[kBatch];
    double kx[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
        const int t = kt0 + tid + u * nthr;
        kp[u] = t < kt1 ? global(S.k_fpos)[t] : 0;
        kx[u] = t < kt1 ? global(kv)[t] : 0.0;
    }
    // The children's update blocks go in rounds (kBatch entries per thread),
    // child after child; the loads of two rounds are in flight ahead of the one
    // being added, the first two issued before the front is cleared.  The
    // records of the current and the next child are read ahead of their rounds.
    const int step = nthr * kBatch;
    struct RoundInfo {   // what the adds of an issued round need
        int child, nc;
        bool first;
        const int32_t* rel;
        const double* uv;
    };
    int pci = c0, pe0 = 0;   // the next round to issue
    ChildRec prec = rec0, pnext = rec1;
    // the fused forward solve's right-hand side of the supernode's columns:
    // the permutation is read before the rounds, thread i's entry of the
    // right-hand side after them (loads complete in the order issued; the
    // right-hand side is waited for where the rounds are about to be added)
    const int pk0 = fw && tid < w ? global(I.perm)[f + tid] : 0;
    auto issue = [&](ChildRound& r, RoundInfo& info) -> bool {
        if (pci >= c1) return false;
        const int nc = prec.nc, ne = (nc * (nc + 1)) / 2;
        const int32_t* rel = S.rel + prec.rel_off;
        const double* uvc = fw ? I.uvec + prec.uv_off : nullptr;
        const bool first = pe0 == 0;
        child_round(U + prec.u_off, rel, nc, ne, pe0, r, first ? uvc : nullptr);
        info = RoundInfo{pci, nc, first, rel, uvc};
        if (pe0 + step < ne) {
            pe0 += step;
        } else {
            ++pci;
            pe0 = 0;
            prec = pnext;
            if (pci + 1 < c1) pnext = child_rec_at(S.child_rec, pci + 1);
        }
        return true;
    };
    ChildRound ra, rb;
    RoundInfo ia{}, ib{};
    bool ha = issue(ra, ia);
    bool hb = issue(rb, ib);
    double rv = 0.0;
    if (fw && tid < w) rv = global(I.rhs)[pk0];
    const int fsize = Lds ? (m * (m + 1)) / 2 : m * (m | 1);
    for (int e = tid; e < fsize; e += nthr) F[e] = 0.0;
    __syncthreads();
    auto place = [&](int pos, double v) {
        if (pos < 0) {
            pos = ~pos;
            v += eta;
        }
        F[pos] = v;
    };
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
        if (kt0 + tid + u * nthr < kt1) place(kp[u], kx[u]);
    for (int t = kt0 + tid + kBatch * nthr; t < kt1; t += nthr) place(global(S.k_fpos)[t], global(kv)[t]);
    // fused forward solve of the Newton step: v over the front's rows starts
    // from the permuted right-hand side of the supernode's columns (before the
    // barrier that precedes the children's update vectors)
    if (fw)
        for (int i = tid; i < m; i += nthr)
            v[i] = i < w ? (i == tid ? rv : global(I.rhs)[global(I.perm)[f + i]]) : 0.0;
    __syncthreads();
    // extend-add in fixed order; children are separated by barriers (two
    // children can add into the same entry, one child's entries are distinct)
    while (ha) {
        ChildRound rc;
        RoundInfo ic{};
        const bool hc = issue(rc, ic);
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (ra.ri[u] >= 0) F[ix(ra.ri[u], ra.rj[u])] += ra.v[u];
        if (fw && ia.first) {   // the child's update vector, with its first round
#pragma unroll
            for (int u = 0; u < kUvec; ++u)
                if (ra.ur[u] >= 0) v[ra.ur[u]] += ra.uv[u];
            for (int i = tid + kUvec * nthr; i < ia.nc; i += nthr) v[ia.rel[i]] += ia.uv[i];
        }
        if (!hb || ib.child != ia.child) __syncthreads();
        ra = rb;
        ia = ib;
        ha = hb;
        rb = rc;
        ib = ic;
        hb = hc;
    }
    partial_cholesky<P>(F, ix, m, w, fail, fw ? v : nullptr, false);
    // the update block (rows and columns w and on) takes its update before the
    // panel goes out: global stores in flight would hold the update's first
    // shared-memory loads until they complete (their data registers are reused)
    if (nb > 0) update_block(F, ix, m, w);
    auto* Ls = global(L + global(S.l_off)[s]);
    for (int jc = wv; jc < w; jc += nw)
        for (int i = lane; i < m; i += kWave) Ls[i + jc * m] = i >= jc ? F[ix(i, jc)] : 0.0;
    if (fw) {   // the forward solve's part of the columns and the update vector
        for (int k = tid; k < w; k += nthr) global(I.xp)[f + k] = v[k];
        auto* us = global(I.uvec + global(S.uv_off)[s]);
        for (int i = w + tid; i < m; i += nthr) us[i - w] = v[i];
    }
    if (nb > 0) {
        auto* Us = global(U + global(S.u_off)[s]);
        for (int jj = wv; jj < nb; jj += nw)
            for (int ii = jj + lane; ii < nb; ii += kWave) Us[ii + jj * nb] = F[ix(w + ii, w + jj)];
    }
    __syncthreads();   // the front buffer is reused by the next supernode of the group
}

// Variants (threads per workgroup, panel width) the autotuner chooses from.
template <bool Lds, int Threads, int P>
__global__ void __launch_bounds__(Threads)
k_factor_groups(const InstPtrs* __restrict__ Ia, const Group* __restrict__ groups, int pred, double eta_force) {
    extern __shared__ double lds[];
    const Group g = groups[blockIdx.x];
    const InstPtrs& I = Ia[g.inst];
    const int s0 = first_node(I, g, pred);
    if (s0 < 0) return;
    const double eta = pred == kPredAll ? eta_force : I.ctl->eta;
    // the front: shared memory, or the instance's global scratch for medium
    // fronts; then the fused forward solve's vector in shared memory
    double* F = Lds ? lds : I.gscratch + (int64_t)g.slot * I.gstride;
    const bool fwd = pred == kPredFactor;   // in a pass: the Newton step's right-hand side is assembled
    for (int i = g.begin; i < g.end; ++i) {
        const int s = i == g.begin ? s0 : I.S.sched_nodes[i];
        const int m = (int)(I.S.rows_ptr[s + 1] - I.S.rows_ptr[s]);
        double* v = Lds ? lds + (m * (m + 1)) / 2 : lds;
        factor_one<Lds, P>(s, I.S, I.kv, eta, I.L, I.U, &I.ctl->fail, F, v, I, fwd);
    }
}

// Forward solve with one supernode's panel P (m x w, column-major, lower w x w
// diagonal block first), staged in shared memory together with the
// reciprocals of its diagonal.  Columns go kPanel at a time: every thread
// solves the small diagonal block itself from broadcast reads, then updates
// the rows it owns; one barrier per block.  v[0:m) holds b; on return xs[0:w) =
// L_dd^{-1} b[0:w) and v[w:m) = b[w:m) - L_below xs.
__device__ __attribute__((always_inline)) void blocked_forward(const double* P, const double* rdiag, int m, int w, double* v, double* xs) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int kb = 0; kb < w; kb += kPanel) {
        const int kw = min(kPanel, w - kb);
        double x[kPanel];
#pragma unroll
        for (int k = 0; k < kPanel; ++k) {
            double s = k < kw ? v[kb + k] : 0.0;
#pragma unroll
            for (int j = 0; j < k; ++j)
                if (k < kw) s = fma(-P[(kb + k) + (int64_t)(kb + j) * m], x[j], s);
            x[k] = k < kw ? s * rdiag[kb + k] : 0.0;
        }
        if (tid < kw) {
#pragma unroll
            for (int k = 0; k < kPanel; ++k)
                if (k == tid) xs[kb + k] = x[k];
        }
        for (int r = kb + kw + tid; r < m; r += nthr) {
            double acc = v[r];
#pragma unroll
            for (int j = 0; j < kPanel; ++j)
                if (j < kw) acc = fma(-P[r + (int64_t)(kb + j) * m], x[j], acc);
            v[r] = acc;
        }
        __syncthreads();
    }
}

// Stage one panel and the reciprocals of its diagonal in shared memory.
__device__ __attribute__((always_inline)) void stage_panel(const double* __restrict__ Ls, int m, int w, double* P, double* rdiag) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    g2s(P, Ls, (int64_t)m * w);
    for (int k = tid; k < w; k += nthr) rdiag[k] = 1.0 / Ls[k + (int64_t)k * m];
}

// Forward substitution L v = P b for one supernode: gather the permuted rhs of
// its columns, add the children's update vectors, solve with the diagonal
// block, then form the update vector of its rows below.
// Shared memory: panel (m w) + rdiag (w) + v (m) + xs (w).
__device__ __attribute__((always_inline)) void fwd_one(int s, const SnView& S, const double* __restrict__ L, double* __restrict__ uvec,
                        const double* __restrict__ rhs, const int32_t* __restrict__ perm, double* __restrict__ xp,
                        double* lds) {
    const int f = S.sn_ptr[s];
    const int w = S.sn_ptr[s + 1] - f;
    const int m = (int)(S.rows_ptr[s + 1] - S.rows_ptr[s]);
    const int tid = threadIdx.x, nthr = blockDim.x;
    double* P = lds;
    double* rdiag = P + (int64_t)m * w;
    double* v = rdiag + w;
    double* xs = v + m;
    stage_panel(L + S.l_off[s], m, w, P, rdiag);
    for (int i = tid; i < m; i += nthr) v[i] = i < w ? rhs[perm[f + i]] : 0.0;
    __syncthreads();
    for (int ci = S.child_ptr[s]; ci < S.child_ptr[s + 1]; ++ci) {
        const int c = S.child_list[ci];
        const int nc = (int)(S.uv_off[c + 1] - S.uv_off[c]);
        const double* uc = uvec + S.uv_off[c];
        const int32_t* rc = S.rel + S.rel_off[c];
        for (int i = tid; i < nc; i += nthr) v[rc[i]] += uc[i];
        __syncthreads();
    }
    blocked_forward(P, rdiag, m, w, v, xs);
    for (int k = tid; k < w; k += nthr) xp[f + k] = xs[k];
    double* us = uvec + S.uv_off[s];
    for (int i = w + tid; i < m; i += nthr) us[i - w] = v[i];
    __syncthreads();
}

__global__ void __launch_bounds__(kFactorBlock)
k_fwd_groups(const InstPtrs* __restrict__ Ia, const Group* __restrict__ groups, int pred, int which) {
    extern __shared__ double lds[];
    const Group g = groups[blockIdx.x];
    const InstPtrs& I = Ia[g.inst];
    const int s0 = first_node(I, g, pred);
    if (s0 < 0) return;
    for (int i = g.begin; i < g.end; ++i)
        fwd_one(i == g.begin ? s0 : I.S.sched_nodes[i], I.S, I.L, I.uvec, solve_in(I, which), I.perm, I.xp, lds);
}

// Value of v in lane k of the wave, in every lane (k wave-uniform).
__device__ __attribute__((always_inline)) inline double lane_value(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// Back substitution L^T x = v for one supernode, after all its ancestors:
// subtract the contribution of the rows below (already final), then solve
// with the transposed diagonal block; writes x unpermuted.  Every global load
// is issued before the first shared-memory store: the diagonal block (staged
// transposed, leading dimension w | 1, kBatch entries per thread per round),
// its diagonal, the supernode's entries of xp, the solution of the rows below
// (gathered through the row list) and the output permutation.  The rows below
// are then read straight from the panel, 16 lanes per column and kBwdCols
// columns per lane group at once (a butterfly sums the lanes).  The diagonal
// block is solved by wave 0, 64 columns at a time from the last: lane j holds
// v_j, x_k leaves lane k through the scalar unit, and the earlier columns take
// the block's contribution before the next block.
// Shared memory: diagonal block (w (w | 1)) + rdiag (w) + xb (m - w) + v (w) + xs (w).
constexpr int kBwdCols = 4;    // columns per 16-lane group in the rows-below product
constexpr int kBwdDepth = 8;   // rows per lane whose loads are in flight together
constexpr int kBwdSub = 16;    // lanes per column in the rows-below product

// Butterfly sums of kBwdCols values over each kBwdSub-lane group, one level for
// all columns at a time so that a level's lane exchanges are in flight together.
__device__ __attribute__((always_inline)) inline void group_sums(double (&acc)[kBwdCols]) {
#pragma unroll
    for (int off = kBwdSub / 2; off > 0; off >>= 1) {
        double x[kBwdCols];
#pragma unroll
        for (int u = 0; u < kBwdCols; ++u) x[u] = __shfl_xor(acc[u], off, kBwdSub);
#pragma unroll
        for (int u = 0; u < kBwdCols; ++u) acc[u] += x[u];
    }
}
__device__ __attribute__((always_inline)) void bwd_one(int s, const SnView& S, const double* __restrict__ L, double* __restrict__ xp,
                        const int32_t* __restrict__ perm, double* __restrict__ out, double* lds) {
    const int f = global(S.sn_ptr)[s];
    const int w = global(S.sn_ptr)[s + 1] - f;
    const int m = (int)(global(S.rows_ptr)[s + 1] - global(S.rows_ptr)[s]);
    const int nb = m - w;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    const int ld = w | 1;
    double* PT = lds;
    double* rdiag = PT + (int64_t)w * ld;
    double* xb = rdiag + w;
    double* v = xb + nb;
    double* xs = v + w;
    const double* Ls = L + global(S.l_off)[s];
    const int32_t* rows = S.rows + global(S.rows_ptr)[s];
    const int ri = tid < nb ? global(rows)[w + tid] : 0;
    const double dg = tid < w ? global(Ls)[tid + (int64_t)tid * m] : 1.0;
    const double xv = tid < w ? global(xp)[f + tid] : 0.0;
    const int pk = tid < w ? global(perm)[f + tid] : 0;
    // rows-below product: 16 lanes per column, kBwdCols columns per lane group;
    // when it takes one pass (w <= kBwdCols * groups, nb <= kSub * kBwdDepth)
    // the panel's values are loaded here, with everything else
    constexpr int kSub = kBwdSub;
    const int sub = tid % kSub, grp = tid / kSub, ngrp = nthr / kSub;
    const bool one_pass = nb > 0 && w <= kBwdCols * ngrp && nb <= kSub * kBwdDepth;
    double lp[kBwdDepth][kBwdCols];
    if (one_pass && grp < w) {
#pragma unroll
        for (int u = 0; u < kBwdCols; ++u) {
            const int jc = grp + u * ngrp;
            const double* col = Ls + (int64_t)(jc < w ? jc : 0) * m + w;
#pragma unroll
            for (int t = 0; t < kBwdDepth; ++t) lp[t][u] = global(col)[min(sub + kSub * t, nb - 1)];
        }
    }
    const int ww = w * w;
    // entry e of the block is (r, c) = (e % w, e / w); the quotient through a
    // single-precision reciprocal is exact here (e < w^2 <= 2^15, and (e + 1/2)
    // / w stays at least 1 / (2 w) away from an integer)
    const float rw = 1.0f / (float)w;
    for (int e0 = 0; e0 < ww; e0 += nthr * kBatch) {
        double t[kBatch];
        int cc[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + tid + u * nthr, c = (int)(((float)e + 0.5f) * rw), r = e - c * w;
            cc[u] = c;
            t[u] = (e < ww && r >= c) ? global(Ls)[r + (int64_t)c * m] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = e0 + tid + u * nthr, c = cc[u], r = e - c * w;
            if (e < ww && r >= c) PT[c + r * ld] = t[u];
        }
    }
    if (tid < nb) xb[tid] = global(xp)[ri];
    if (tid < w) {
        rdiag[tid] = 1.0 / dg;
        v[tid] = xv;
    }
    // the panel fits in shared memory, so w < nthr; a narrow supernode can have
    // more rows below than threads
    for (int i = tid + nthr; i < nb; i += nthr) xb[i] = global(xp)[global(rows)[w + i]];
    for (int k = tid + nthr; k < w; k += nthr) {
        rdiag[k] = 1.0 / global(Ls)[k + (int64_t)k * m];
        v[k] = global(xp)[f + k];
    }
    __syncthreads();
    if (one_pass) {
        if (grp < w) {   // uniform over each 16-lane group
            double acc[kBwdCols];
#pragma unroll
            for (int u = 0; u < kBwdCols; ++u) acc[u] = 0.0;
#pragma unroll
            for (int t = 0; t < kBwdDepth; ++t) {
                const int i = sub + kSub * t;
                const double xv = i < nb ? xb[min(i, nb - 1)] : 0.0;
#pragma unroll
                for (int u = 0; u < kBwdCols; ++u) acc[u] = fma(lp[t][u], xv, acc[u]);
            }
            group_sums(acc);
#pragma unroll
            for (int u = 0; u < kBwdCols; ++u) {
                const int jc = grp + u * ngrp;
                if (sub == 0 && jc < w) v[jc] -= acc[u];
            }
        }
    } else
    for (int jc0 = grp; jc0 < w; jc0 += kBwdCols * ngrp) {
        double acc[kBwdCols];
        const double* col[kBwdCols];
#pragma unroll
        for (int u = 0; u < kBwdCols; ++u) {
            const int jc = jc0 + u * ngrp;
            acc[u] = 0.0;
            col[u] = Ls + (int64_t)(jc < w ? jc : 0) * m + w;
        }
        // kBwdDepth rows per lane at a time, all their loads issued together
        // (rows past nb load row nb - 1 and add zero; a column past w reads
        // column 0 and is not stored)
        for (int i0 = sub; i0 < nb; i0 += kSub * kBwdDepth) {
            double lv[kBwdDepth][kBwdCols], xv[kBwdDepth];
#pragma unroll
            for (int t = 0; t < kBwdDepth; ++t) {
                const int i = i0 + kSub * t, ic = min(i, nb - 1);
                xv[t] = i < nb ? xb[ic] : 0.0;
#pragma unroll
                for (int u = 0; u < kBwdCols; ++u) lv[t][u] = global(col[u])[ic];
            }
#pragma unroll
            for (int t = 0; t < kBwdDepth; ++t)
#pragma unroll
                for (int u = 0; u < kBwdCols; ++u) acc[u] = fma(lv[t][u], xv[t], acc[u]);
        }
        group_sums(acc);
#pragma unroll
        for (int u = 0; u < kBwdCols; ++u) {
            const int jc = jc0 + u * ngrp;
            if (sub == 0 && jc < w) v[jc] -= acc[u];
        }
    }
    __syncthreads();
    for (int b0 = ((w - 1) / kWave) * kWave; b0 >= 0; b0 -= kWave) {
        const int bw = min(kWave, w - b0);
        if (wv == 0) {
            const int j = lane;
            double vj = j < bw ? v[b0 + j] : 0.0;
#pragma unroll
            for (int k = kWave - 1; k >= 0; --k) {
                if (k < bw) {   // wave-uniform
                    const double xk = lane_value(vj, k) * rdiag[b0 + k];
                    const double upd = fma(-PT[(b0 + j) + (b0 + k) * ld], xk, vj);
                    vj = j == k ? xk : (j < k ? upd : vj);
                }
            }
            if (j < bw) xs[b0 + j] = vj;
        }
        __syncthreads();
        if (b0 > 0) {   // columns before the block: v[c] -= L(block, c)^T x(block)
            for (int c = tid; c < b0; c += nthr) {
                double acc = v[c];
                for (int q = 0; q < bw; ++q) acc = fma(-PT[c + (b0 + q) * ld], xs[b0 + q], acc);
                v[c] = acc;
            }
            __syncthreads();
        }
    }
    if (tid < w) {
        global(xp)[f + tid] = xs[tid];
        global(out)[pk] = xs[tid];
    }
    for (int k = tid + nthr; k < w; k += nthr) {
        global(xp)[f + k] = xs[k];
        global(out)[global(perm)[f + k]] = xs[k];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kFactorBlock)
k_bwd_groups(const InstPtrs* __restrict__ Ia, const Group* __restrict__ groups, int pred, int which) {
    extern __shared__ double lds[];
    const Group g = groups[blockIdx.x];
    const InstPtrs& I = Ia[g.inst];
    const int s0 = first_node(I, g, pred);
    if (s0 < 0) return;
    for (int i = g.begin; i < g.end; ++i)
        bwd_one(i == g.begin ? s0 : I.S.sched_nodes[i], I.S, I.L, I.xp, I.perm, solve_out(I, which), lds);
}

}  // namespace

hipError_t linalg_configure(size_t max_lds_bytes) {
    const void* fns[] = {reinterpret_cast<const void*>(k_factor_groups<true, 256, 8>),
                         reinterpret_cast<const void*>(k_factor_groups<true, 512, 8>),
                         reinterpret_cast<const void*>(k_factor_groups<true, 128, 8>),
                         reinterpret_cast<const void*>(k_factor_groups<true, 256, 4>),
                         reinterpret_cast<const void*>(k_factor_groups<true, 512, 4>),
                         reinterpret_cast<const void*>(k_fwd_groups), reinterpret_cast<const void*>(k_bwd_groups)};
    for (const void* fn : fns) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int Threads, int P>
void launch_variant(bool lds, int pred, double eta_force, const InstPtrs* I, const Group* g, int groups,
                    size_t lds_bytes, hipStream_t st) {
    if (lds)
        hipLaunchKernelGGL((k_factor_groups<true, Threads, P>), dim3(groups), dim3(Threads), lds_bytes, st, I, g, pred,
                           eta_force);
    else
        hipLaunchKernelGGL((k_factor_groups<false, Threads, P>), dim3(groups), dim3(Threads),
                           kMediumFront * sizeof(double), st, I, g, pred, eta_force);
}

void launch_factor_groups(bool lds, int variant, int pred, double eta_force, const InstPtrs* I, const Group* g,
                          int groups, size_t lds_bytes, hipStream_t st) {
    if (groups <= 0) return;
    switch (variant) {
        case 1: launch_variant<512, 8>(lds, pred, eta_force, I, g, groups, lds_bytes, st); break;
        case 2: launch_variant<128, 8>(lds, pred, eta_force, I, g, groups, lds_bytes, st); break;
        case 3: launch_variant<256, 4>(lds, pred, eta_force, I, g, groups, lds_bytes, st); break;
        case 4: launch_variant<512, 4>(lds, pred, eta_force, I, g, groups, lds_bytes, st); break;
        default: launch_variant<256, 8>(lds, pred, eta_force, I, g, groups, lds_bytes, st); break;
    }
}

void launch_fwd_groups(int pred, int which, const InstPtrs* I, const Group* g, int groups, size_t lds_bytes,
                       hipStream_t st) {
    if (groups <= 0) return;
    hipLaunchKernelGGL(k_fwd_groups, dim3(groups), dim3(kFactorBlock), lds_bytes, st, I, g, pred, which);
}

void launch_bwd_groups(int pred, int which, const InstPtrs* I, const Group* g, int groups, size_t lds_bytes,
                       hipStream_t st) {
    if (groups <= 0) return;
    hipLaunchKernelGGL(k_bwd_groups, dim3(groups), dim3(kFactorBlock), lds_bytes, st, I, g, pred, which);
}

}  // namespace nmpc
