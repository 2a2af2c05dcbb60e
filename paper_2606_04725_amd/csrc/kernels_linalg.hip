// Numeric supernodal Cholesky and triangular solves (eqs. 20-25), multifrontal
// form: supernode s owns a dense front F_s of size m_s x m_s over its row list
// R_s (its w_s own columns first).  F_s starts from the KKT entries of its
// columns, receives the update blocks of its children by extend-add through
// precomputed relative positions, and is partially factored on its first w_s
// columns; the factored columns are the L panel (eq. 21 restricted to S_L) and
// the trailing block is the update passed to the parent.  One workgroup per
// supernode, one launch per level of the supernodal elimination tree; every
// sum is taken in a fixed order, so results do not depend on scheduling.
#include <cmath>

#include "kernels.h"

namespace nmpc {

namespace {

// Right-looking partial Cholesky of the first w columns of an m x m front
// (column-major, lower triangle).  Pivot columns are taken kPanel at a time:
// the panel is factored column by column, then the rest of the front is
// updated with 4 x 4 register tiles.  A pivot that is not positive and finite
// sets *fail (the matrix is not numerically positive definite, eq. 12).
__device__ void partial_cholesky(double* F, int m, int w, int* fail) {
    const int tid = threadIdx.x;
    for (int kb = 0; kb < w; kb += kPanel) {
        const int kw = min(kPanel, w - kb);
        for (int k = kb; k < kb + kw; ++k) {
            double piv = F[k + (int64_t)k * m];
            if (!(piv > 0.0) || !(piv < INFINITY)) {
                if (tid == 0) *fail = 1;
                piv = 1.0;
            }
            const double sq = sqrt(piv);
            const double inv = 1.0 / sq;
            for (int i = k + 1 + tid; i < m; i += blockDim.x) F[i + (int64_t)k * m] *= inv;
            __syncthreads();
            if (tid == 0) F[k + (int64_t)k * m] = sq;
            const int ncol = kb + kw - (k + 1);
            const int nr = m - (k + 1);
            if (ncol > 0) {
                for (int e = tid; e < ncol * nr; e += blockDim.x) {
                    const int jj = e / nr, ii = e - jj * nr;
                    const int jc = k + 1 + jj, ir = k + 1 + ii;
                    if (ir >= jc) F[ir + (int64_t)jc * m] -= F[ir + (int64_t)k * m] * F[jc + (int64_t)k * m];
                }
            }
            __syncthreads();
        }
        const int t0 = kb + kw;
        const int T = m - t0;
        if (T > 0) {
            const int nt = (T + 3) / 4;
            const int ntiles = nt * (nt + 1) / 2;
            for (int tile = tid; tile < ntiles; tile += blockDim.x) {
                int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
                while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
                while (ti * (ti + 1) / 2 > tile) --ti;
                const int tj = tile - ti * (ti + 1) / 2;
                const int i0 = t0 + 4 * ti, j0 = t0 + 4 * tj;
                double acc[4][4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
                for (int k = kb; k < t0; ++k) {
                    double av[4], bv[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        av[r] = (i0 + r < m) ? F[i0 + r + (int64_t)k * m] : 0.0;
                        bv[r] = (j0 + r < m) ? F[j0 + r + (int64_t)k * m] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[r][q] = fma(av[r], bv[q], acc[r][q]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int ir = i0 + r, jc = j0 + q;
                        if (ir < m && jc < m && ir >= jc) F[ir + (int64_t)jc * m] -= acc[r][q];
                    }
            }
        }
        __syncthreads();
    }
}

template <bool Lds>
__global__ void __launch_bounds__(kFactorBlock)
k_factor_level(const int32_t* __restrict__ nodes, SnView S, const double* __restrict__ kv, double eta,
               double* __restrict__ L, double* __restrict__ U, int* __restrict__ fail,
               double* __restrict__ gscratch, int64_t gstride) {
    extern __shared__ double lds[];
    const int s = nodes[blockIdx.x];
    const int f = S.sn_ptr[s];
    const int w = S.sn_ptr[s + 1] - f;
    const int m = (int)(S.rows_ptr[s + 1] - S.rows_ptr[s]);
    const int nb = m - w;
    const int tid = threadIdx.x;
    double* F = Lds ? lds : gscratch + (int64_t)blockIdx.x * gstride;
    const int64_t mm = (int64_t)m * m;
    for (int64_t e = tid; e < mm; e += blockDim.x) F[e] = 0.0;
    __syncthreads();
    // original entries of the condensed matrix in this supernode's columns (+ eta I)
    for (int t = S.k_ptr[s] + tid; t < S.k_ptr[s + 1]; t += blockDim.x) {
        const int pos = S.k_fpos[t];
        double v = kv[t];
        if (pos % (m + 1) == 0) v += eta;
        F[pos] = v;
    }
    __syncthreads();
    // extend-add of the children's update blocks, children in fixed order
    for (int ci = S.child_ptr[s]; ci < S.child_ptr[s + 1]; ++ci) {
        const int c = S.child_list[ci];
        const int wc = S.sn_ptr[c + 1] - S.sn_ptr[c];
        const int nc = (int)(S.rows_ptr[c + 1] - S.rows_ptr[c]) - wc;
        const double* Uc = U + S.u_off[c];
        const int32_t* rc = S.rel + S.rel_off[c];
        const int64_t tot = (int64_t)nc * nc;
        for (int64_t e = tid; e < tot; e += blockDim.x) {
            const int jj = (int)(e / nc), ii = (int)(e - (int64_t)jj * nc);
            if (ii >= jj) F[rc[ii] + (int64_t)rc[jj] * m] += Uc[ii + (int64_t)jj * nc];
        }
        __syncthreads();
    }
    partial_cholesky(F, m, w, fail);
    // factored columns -> L panel, trailing block -> update for the parent
    double* Ls = L + S.l_off[s];
    const int64_t lw = (int64_t)m * w;
    for (int64_t e = tid; e < lw; e += blockDim.x) Ls[e] = F[e];
    if (nb > 0) {
        double* Us = U + S.u_off[s];
        const int64_t tot = (int64_t)nb * nb;
        for (int64_t e = tid; e < tot; e += blockDim.x) {
            const int jj = (int)(e / nb), ii = (int)(e - (int64_t)jj * nb);
            Us[e] = F[(w + ii) + (int64_t)(w + jj) * m];
        }
    }
}

// Forward substitution L v = P b for one supernode: gather the permuted rhs
// of its columns, add the children's update vectors, solve with the diagonal
// block and form the update vector of its rows below.
template <bool Stage>
__global__ void __launch_bounds__(kFactorBlock)
k_fwd_level(const int32_t* __restrict__ nodes, SnView S, const double* __restrict__ L,
            double* __restrict__ uvec, const double* __restrict__ rhs, const int32_t* __restrict__ perm,
            double* __restrict__ xp) {
    extern __shared__ double lds[];
    const int s = nodes[blockIdx.x];
    const int f = S.sn_ptr[s];
    const int w = S.sn_ptr[s + 1] - f;
    const int m = (int)(S.rows_ptr[s + 1] - S.rows_ptr[s]);
    const int tid = threadIdx.x;
    const double* Ls = L + S.l_off[s];
    const int64_t lw = (int64_t)m * w;
    double* v = Stage ? lds + lw : lds;     // m
    if (Stage)
        for (int64_t e = tid; e < lw; e += blockDim.x) lds[e] = Ls[e];
    const double* P = Stage ? lds : Ls;     // m x w panel
    for (int i = tid; i < m; i += blockDim.x) v[i] = i < w ? rhs[perm[f + i]] : 0.0;
    __syncthreads();
    for (int ci = S.child_ptr[s]; ci < S.child_ptr[s + 1]; ++ci) {
        const int c = S.child_list[ci];
        const int nc = (int)(S.uv_off[c + 1] - S.uv_off[c]);
        const double* uc = uvec + S.uv_off[c];
        const int32_t* rc = S.rel + S.rel_off[c];
        for (int i = tid; i < nc; i += blockDim.x) v[rc[i]] += uc[i];
        __syncthreads();
    }
    for (int k = 0; k < w; ++k) {
        const double xk = v[k] / P[k + (int64_t)k * m];
        if (tid == 0) xp[f + k] = xk;
        for (int i = k + 1 + tid; i < m; i += blockDim.x) v[i] -= P[i + (int64_t)k * m] * xk;
        __syncthreads();
    }
    const int nb = m - w;
    double* us = uvec + S.uv_off[s];
    for (int i = tid; i < nb; i += blockDim.x) us[i] = v[w + i];
}

// Back substitution L^T x = v for one supernode, after all its ancestors:
// subtract the contribution of the rows below (already final), then solve
// with the transposed diagonal block; writes x unpermuted.
template <bool Stage>
__global__ void __launch_bounds__(kFactorBlock)
k_bwd_level(const int32_t* __restrict__ nodes, SnView S, const double* __restrict__ L,
            double* __restrict__ xp, const int32_t* __restrict__ perm, double* __restrict__ out) {
    extern __shared__ double lds[];
    const int s = nodes[blockIdx.x];
    const int f = S.sn_ptr[s];
    const int w = S.sn_ptr[s + 1] - f;
    const int m = (int)(S.rows_ptr[s + 1] - S.rows_ptr[s]);
    const int nb = m - w;
    const int tid = threadIdx.x;
    const double* Ls = L + S.l_off[s];
    const int64_t lw = (int64_t)m * w;
    double* xb = Stage ? lds + lw : lds;
    double* v = xb + nb;
    if (Stage)
        for (int64_t e = tid; e < lw; e += blockDim.x) lds[e] = Ls[e];
    const double* P = Stage ? lds : Ls;
    const int32_t* rows = S.rows + S.rows_ptr[s];
    for (int i = tid; i < nb; i += blockDim.x) xb[i] = xp[rows[w + i]];
    __syncthreads();
    for (int jc = tid; jc < w; jc += blockDim.x) {
        double acc = xp[f + jc];
        for (int i = 0; i < nb; ++i) acc -= P[(w + i) + (int64_t)jc * m] * xb[i];
        v[jc] = acc;
    }
    __syncthreads();
    for (int k = w - 1; k >= 0; --k) {
        const double xk = v[k] / P[k + (int64_t)k * m];
        if (tid == 0) {
            xp[f + k] = xk;
            out[perm[f + k]] = xk;
        }
        for (int jc = tid; jc < k; jc += blockDim.x) v[jc] -= P[k + (int64_t)jc * m] * xk;
        __syncthreads();
    }
}

}  // namespace

hipError_t linalg_configure(size_t max_lds_bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_factor_level<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_fwd_level<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_bwd_level<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds_bytes);
}

void launch_factor_level(bool lds, const int32_t* nodes, int count, size_t lds_bytes, const SnView& S,
                         const double* kv, double eta, double* L, double* U, int* fail, double* gscratch,
                         int64_t gstride, hipStream_t st) {
    if (count <= 0) return;
    if (lds)
        hipLaunchKernelGGL(k_factor_level<true>, dim3(count), dim3(kFactorBlock), lds_bytes, st, nodes, S, kv,
                           eta, L, U, fail, gscratch, gstride);
    else
        hipLaunchKernelGGL(k_factor_level<false>, dim3(count), dim3(kFactorBlock), 0, st, nodes, S, kv, eta, L,
                           U, fail, gscratch, gstride);
}

void launch_fwd_level(bool stage, const int32_t* nodes, int count, size_t lds_bytes, const SnView& S,
                      const double* L, double* uvec, const double* rhs, const int32_t* perm, double* xp,
                      hipStream_t st) {
    if (count <= 0) return;
    if (stage)
        hipLaunchKernelGGL(k_fwd_level<true>, dim3(count), dim3(kFactorBlock), lds_bytes, st, nodes, S, L, uvec,
                           rhs, perm, xp);
    else
        hipLaunchKernelGGL(k_fwd_level<false>, dim3(count), dim3(kFactorBlock), lds_bytes, st, nodes, S, L,
                           uvec, rhs, perm, xp);
}

void launch_bwd_level(bool stage, const int32_t* nodes, int count, size_t lds_bytes, const SnView& S,
                      const double* L, double* xp, const int32_t* perm, double* out, hipStream_t st) {
    if (count <= 0) return;
    if (stage)
        hipLaunchKernelGGL(k_bwd_level<true>, dim3(count), dim3(kFactorBlock), lds_bytes, st, nodes, S, L, xp,
                           perm, out);
    else
        hipLaunchKernelGGL(k_bwd_level<false>, dim3(count), dim3(kFactorBlock), lds_bytes, st, nodes, S, L, xp,
                           perm, out);
}

}  // namespace nmpc
