// Dense partial Cholesky of a front held in shared memory, shared by the
// small-front kernels and the diagonal blocks of the large-front path.
#pragma once

#include <cmath>

namespace nmpc {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kCholWave = 64;

// Index maps of a front's lower triangle: base(j) + i is the position of
// entry (i, j), i >= j.  Front orders stay far below 2^12, so the products
// fit the full-rate 24-bit multiplier.
struct SquareIdx {   // column-major, leading dimension ld
    int ld;
    __device__ int base(int j) const { return __mul24(j, ld); }
    __device__ int operator()(int i, int j) const { return i + base(j); }
};
struct PackedIdx {   // lower triangle packed by columns: column j holds rows j .. m-1
    int m;
    __device__ int base(int j) const { return __mul24(j, m) - (__mul24(j, j + 1) >> 1); }
    __device__ int operator()(int i, int j) const { return base(j) + i; }
};

// Tiles of a lower trapezoid of nt tile rows and nc <= nt tile columns, in
// row order: the triangle of the first nc rows, then nc tiles per row.
__device__ inline int tile_count(int nt, int nc) { return (__mul24(nc, nc + 1) >> 1) + __mul24(nt - nc, nc); }
__device__ inline void tile_of(int tt, int nc, int& ti, int& tj) {
    const int tri = __mul24(nc, nc + 1) >> 1;
    if (tt < tri) {   // tile row ti holds tiles ti (ti + 1) / 2 ...: single-precision root, integer correction
        ti = (int)((sqrtf(8.0f * (float)tt + 1.0f) - 1.0f) * 0.5f);
        while ((__mul24(ti + 1, ti + 2) >> 1) <= tt) ++ti;
        while ((__mul24(ti, ti + 1) >> 1) > tt) --ti;
        tj = tt - (__mul24(ti, ti + 1) >> 1);
    } else {
        const int r = tt - tri;
        ti = nc + r / nc;
        tj = r - __mul24(ti - nc, nc);
    }
}

// Steps 1 and 2 of pivot columns [kb, kb + kw), kw <= P (a full panel is
// called with kw = P as a constant, so its bounds checks fold away): d gets
// the factored P x P pivot block and, with fv, xk the panel's part of the
// forward solve, in the registers of every thread that takes part (waves that
// own a row below the block, and wave 0, which stores both); the others would
// repeat the block's factorization for nothing on a SIMD that a working wave
// shares.
template <int P, class Idx>
__device__ __attribute__((always_inline)) inline void panel_solve(double* F, Idx ix, int m, int kb, int kw, int* fail,
                                                                 double* fv, double (&d)[P][P], double (&xk)[P]) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wv = tid / kCholWave;
    if (!(wv == 0 || kb + kw + wv * kCholWave < m)) return;
    double rinv[P], rd[P];
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
        for (int j = 0; j < P; ++j)
            d[i][j] = (j <= i && i < kw) ? F[ix(kb + i, kb + j)] : (i == j ? 1.0 : 0.0);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double piv = d[k][k];
        if (k < kw && (!(piv > 0.0) || !(piv < INFINITY))) {
            bad = true;
            piv = 1.0;
        }
        // one reciprocal square root per pivot: d_kk = piv / sqrt(piv), and the
        // reciprocal doubles as the row solves' 1 / d_kk
        const double inv = rsqrt(piv);
        rinv[k] = inv;
        d[k][k] = piv * inv;
#pragma unroll
        for (int i = k + 1; i < P; ++i) d[i][k] *= inv;
#pragma unroll
        for (int j = k + 1; j < P; ++j)
#pragma unroll
            for (int i = j; i < P; ++i) d[i][j] = fma(-d[i][k], d[j][k], d[i][j]);
    }
    if (bad && tid == 0) *fail = 1;
#pragma unroll
    for (int k = 0; k < P; ++k) rd[k] = k < kw ? rinv[k] : 1.0;
    if (fv) {   // fv[kb, kb + kw) is final: every earlier panel updated it at least one barrier ago
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double acc = k < kw ? fv[kb + k] : 0.0;
#pragma unroll
            for (int j = 0; j < k; ++j) acc = fma(-d[k][j], xk[j], acc);
            xk[k] = k < kw ? acc * rd[k] : 0.0;
        }
    }
    // step 2 follows at once: it reads only rows below the block, and the
    // factored block is stored after the next barrier, when every wave has
    // read the block's original entries
    for (int r = kb + kw + tid; r < m; r += nthr) {
        double a[P];
#pragma unroll
        for (int j = 0; j < P; ++j) a[j] = j < kw ? F[ix(r, kb + j)] : 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double s = a[k];
#pragma unroll
            for (int j = 0; j < k; ++j) s = fma(-a[j], d[k][j], s);
            a[k] = s * rd[k];
        }
#pragma unroll
        for (int j = 0; j < P; ++j)
            if (j < kw) F[ix(r, kb + j)] = a[j];
        if (fv) {
            double acc = fv[r];
#pragma unroll
            for (int j = 0; j < P; ++j) acc = fma(-a[j], xk[j], acc);
            fv[r] = acc;
        }
    }
}

// The factored pivot block into the front by thread 0 (every value is in its
// registers): per column one base address, then the column's entries at
// constant offsets from it, all under one branch.  With fv, the panel's part
// of the forward solve replaces its right-hand side there (every wave that
// read that right-hand side has passed the barrier before this call).
template <int P, class Idx>
__device__ __attribute__((always_inline)) inline void store_pivot_block(double* F, Idx ix, int kb, int kw,
                                                                       const double (&d)[P][P], double* fv,
                                                                       const double (&xk)[P]) {
    if (threadIdx.x != 0) return;
    if (fv) {
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (k < kw) fv[kb + k] = xk[k];
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        if (j >= kw) break;
        double* col = F + ix(kb, kb + j);   // entry (kb + i, kb + j) is col[i]
#pragma unroll
        for (int i = j; i < P; ++i)
            if (i < kw) col[i] = d[i][j];
    }
}

// Step 3 on one 16 x 16 tile (ti, tj) of the lower trapezoid right of and
// below pivot columns [kb, kb + kw): rows [t0, m), columns [t0, w), t0 = kb +
// kw.  One v_mfma_f64_16x16x4f64 per 4 pivot columns.
template <int P, class Idx>
__device__ __attribute__((always_inline)) inline void trapezoid_tile(double* F, Idx ix, int m, int w, int kb, int kw,
                                                                    int ti, int tj) {
    const int lane = threadIdx.x & (kCholWave - 1), li = lane & 15, lk = lane >> 4;
    const int t0 = kb + kw, i0 = t0 + 16 * ti, j0 = t0 + 16 * tj;
    // every operand is loaded from an entry inside the front (rows and pivot
    // columns clamped) and zeroed afterwards where it lies outside, so the
    // loads need no branch
    const bool va = i0 + li < m, vb = j0 + li < w;
    const int ra = va ? i0 + li : m - 1, rb = vb ? j0 + li : w - 1;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    double av[P / 4], bv[P / 4];
#pragma unroll
    for (int s4 = 0; s4 < P / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        const double* col = F + ix.base(kb + (kk < kw ? kk : kw - 1));
        av[s4] = col[ra];
        bv[s4] = col[rb];
    }
#pragma unroll
    for (int s4 = 0; s4 < P / 4; ++s4) {
        const bool in = 4 * s4 + lk < kw;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(in && va ? av[s4] : 0.0, in && vb ? bv[s4] : 0.0, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ir = i0 + 4 * r + lk, jc = j0 + li;
        if (ir < m && jc <= ir && jc < w) F[ix(ir, jc)] -= acc[r];
    }
}

// The update block of the front (rows and columns [w, m)) minus L21 L21^T,
// L21 = the panel's rows [w, m): lower-triangle 16 x 16 tiles over the waves,
// one v_mfma_f64_16x16x4f64 per 4 panel columns, each entry read and written
// once.
template <class Idx>
__device__ __attribute__((always_inline)) inline void update_block(double* F, Idx ix, int m, int w) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & (kCholWave - 1), wv = tid / kCholWave, nw = nthr / kCholWave;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (m - w + 15) / 16;
    for (int tt = wv; tt < tile_count(nt, nt); tt += nw) {
        int ti, tj;
        tile_of(tt, nt, ti, tj);
        const int i0 = w + 16 * ti, j0 = w + 16 * tj;
        // rows clamped into the front and zeroed after the load (no branch
        // around the loads); the steps whose four columns all lie below w
        // run without a column check, the last step clamps its columns too
        const bool va = i0 + li < m, vb = j0 + li < m;
        const int ra = va ? i0 + li : m - 1, rb = vb ? j0 + li : m - 1;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        const int wfull = w & ~3;
        int k4 = 0;
        for (; k4 + 16 <= wfull; k4 += 16) {   // four steps: eight loads in flight, then the products
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double* col = F + ix.base(k4 + 4 * u + lk);
                a[u] = col[ra];
                b[u] = col[rb];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va ? a[u] : 0.0, vb ? b[u] : 0.0, acc, 0, 0, 0);
        }
        for (; k4 < wfull; k4 += 4) {
            const double* col = F + ix.base(k4 + lk);
            const double a = col[ra], b = col[rb];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va ? a : 0.0, vb ? b : 0.0, acc, 0, 0, 0);
        }
        if (k4 < w) {
            const int kk = k4 + lk;
            const double* col = F + ix.base(kk < w ? kk : w - 1);
            const double a = col[ra], b = col[rb];
            const bool in = kk < w;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(in && va ? a : 0.0, in && vb ? b : 0.0, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ir = i0 + 4 * r + lk, jc = j0 + li;
            if (ir < m && jc <= ir) F[ix(ir, jc)] -= acc[r];
        }
    }
    __syncthreads();
}

// Right-looking partial Cholesky of the first w columns of an m x m front
// (lower triangle, positions given by the index map ix; only entries i >= j are
// touched), P pivot columns at a time:
//  1. every thread of a wave that owns rows below the block (and of wave 0)
//     factors the P x P diagonal block itself, in registers (identical
//     arithmetic in every such thread, no communication);
//  2. every row below the block solves its own row of the panel against it;
//  3. the panel's remaining columns take the rank-P update on the matrix
//     cores in 16 x 16 tiles: first the tile column holding the next pivot
//     columns (P <= 16), then, after a barrier, the other tiles on the waves
//     that have no rows of the next panel, while the waves that do run steps
//     1 and 2 of the next panel (the two touch different columns);
// and after the last panel the update block (rows and columns w and on) takes
// the rank-w update of all panel columns at once (unless the caller does so
// itself, with_update = false, e.g. to store the panel meanwhile).
// A pivot that is not positive and finite sets *fail (eq. 12: the matrix is not
// numerically positive definite); the arithmetic continues with pivot 1.
// With fv, a forward substitution rides along: fv (shared memory, m values)
// holds the right-hand side over the front's rows; each panel's x = D^{-1}
// fv[panel] is formed from the registers holding D, every row below takes
// fv[r] -= L[r, panel] x in step 2, and x replaces fv[panel] with the pivot
// block's store.  On return (after a barrier) fv[0, w) holds the solution of
// the front's columns and fv[w, m) the update vector of the rows below; the
// caller writes them out (global stores here would hold up the next shared-
// memory loads that reuse their registers).
template <int P, class Idx>
__device__ __attribute__((always_inline)) inline void partial_cholesky(double* F, Idx ix, int m, int w, int* fail, double* fv = nullptr,
                                        bool with_update = true) {
    static_assert(P % 4 == 0 && P <= 16, "the next pivot columns lie in the first tile column");
    const int wv = threadIdx.x / kCholWave, nw = blockDim.x / kCholWave;
    double d[P][P], xk[P];
    if (w >= P)
        panel_solve<P>(F, ix, m, 0, P, fail, fv, d, xk);
    else if (w > 0)
        panel_solve<P>(F, ix, m, 0, w, fail, fv, d, xk);
    for (int kb = 0; kb < w; kb += P) {   // steps 1 and 2 of panel kb are done
        const int kw = min(P, w - kb), t0 = kb + kw;
        const int nt = (m - t0 + 15) / 16, nc = (w - t0 + 15) / 16;
        __syncthreads();
        if (kw == P)   // a full panel: the width is a constant and the stores need no bounds
            store_pivot_block<P>(F, ix, kb, P, d, fv, xk);
        else
            store_pivot_block<P>(F, ix, kb, kw, d, fv, xk);
        if (t0 < w)
            for (int ti = wv; ti < nt; ti += nw) trapezoid_tile<P>(F, ix, m, w, kb, kw, ti, 0);
        __syncthreads();
        if (t0 < w) {
            const int kw2 = min(P, w - t0);
            // waves with rows of the next panel (wave 0 always takes part)
            const int busy = min(nw, max(1, (m - t0 - kw2 + kCholWave - 1) / kCholWave));
            const int rest = tile_count(nt - 1, nc - 1);
            const int first = busy < nw ? wv - busy : wv, stride = busy < nw ? nw - busy : nw;
            if (first >= 0)
                for (int tt = first; tt < rest; tt += stride) {
                    int ti, tj;
                    tile_of(tt, nc - 1, ti, tj);
                    trapezoid_tile<P>(F, ix, m, w, kb, kw, ti + 1, tj + 1);
                }
            if (kw2 == P)
                panel_solve<P>(F, ix, m, t0, P, fail, fv, d, xk);
            else
                panel_solve<P>(F, ix, m, t0, kw2, fail, fv, d, xk);
        }
    }
    if (with_update && m > w) update_block(F, ix, m, w);
}

}  // namespace nmpc
