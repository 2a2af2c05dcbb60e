// Large supernodes: numeric factorization and solves (eqs. 20-25) spread over
// many workgroups.  A front that does not fit in shared memory is assembled
// and factored in place in its final storage: column j < w of the front is
// column j of the supernode's L panel (m x w, leading dimension m) and the
// trailing block is the update block handed to the parent ((m - w) x (m - w),
// leading dimension m - w).  Every launch covers one step for all large
// supernodes of one tree level (of every instance of a batch), described by a
// task list; every sum is taken in a fixed order, so results do not depend on
// how tasks are scheduled.
//
// Factorization of one level: zero the fronts and scatter the KKT entries
// (+ eta on the diagonal); add the children's update blocks, one child per
// launch; then per outer panel of kBigOuter columns, per inner panel of
// kBigPanel columns: factor the diagonal block (one workgroup per front), solve
// the rows below it (rows split over workgroups), and update the rest of the
// outer panel; then one rank-kBigOuter update of the trailing lower triangle.
// Updates run on the matrix cores (64 x 64 tiles over workgroups, one
// v_mfma_f64_16x16x4f64 per 4 columns); the outer panel keeps the update
// blocks' read-modify-write traffic to one pass per kBigOuter columns.
//
// Solves: forward, one workgroup gathers the right-hand side and the children's
// update vectors and solves with the diagonal block, then the rows below are a
// GEMV split over workgroups; backward, the transposed GEMV with the rows below
// is split over column blocks, then one workgroup solves with the transposed
// diagonal block.
#include <cmath>

#include "kernels.h"
#include "front_chol.h"

namespace nmpc {

namespace {

constexpr int kWave = 64;
constexpr int kRowBlock = kBlock / 4;   // TRSM rows per workgroup (four lanes per row)
constexpr int kTile = 64;        // trailing-update tile
constexpr int kSolveRows = 256;  // GEMV rows per workgroup
constexpr int kSolveCols = 16;   // transposed-GEMV columns per workgroup
constexpr int kTri = kWave * (kWave + 1);   // a staged 64 x 64 triangle, leading dimension 65
constexpr int kStage = kWave * kWave / kBlock;   // entries of a 64 x 64 block staged per thread
constexpr int kUpdateDepth = 8;  // 4-column steps of an update tile whose loads are in flight together
constexpr int kExtendDepth = 4;  // child rows per thread whose loads are in flight together

struct Front {
    double* L;     // panel, leading dimension m
    double* U;     // update block, leading dimension m - w
    int f, w, m;
};

__device__ inline Front front_of(const InstPtrs& I, int s) {
    Front F;
    F.f = I.S.sn_ptr[s];
    F.w = I.S.sn_ptr[s + 1] - F.f;
    F.m = (int)(I.S.rows_ptr[s + 1] - I.S.rows_ptr[s]);
    F.L = I.L + I.S.l_off[s];
    F.U = I.U + I.S.u_off[s];
    return F;
}

// address of front entry (i, j), i >= j
__device__ inline double* at(const Front& F, int i, int j) {
    return j < F.w ? F.L + i + (int64_t)j * F.m : F.U + (i - F.w) + (int64_t)(j - F.w) * (F.m - F.w);
}

// Fused forward substitution of the Newton step (eq. 23), run by the
// factorization of a supernode whose whole subtree runs it: the vector over
// the front's rows starts as the permuted right-hand side of its columns plus
// the children's update vectors; each panel's solution replaces its entries,
// and the rows below take the panel's product as their rows are solved.
// Entry i lives in xp (i < w) or in the supernode's update vector (i >= w),
// where the unfused solve leaves them too.
__device__ inline bool fwd_fused(const InstPtrs& I, int s, int pred) { return pred == kPredFactor && I.S.fused[s]; }
__device__ inline double* fwd_entry(const InstPtrs& I, const Front& F, int s, int i) {
    return i < F.w ? I.xp + F.f + i : I.uvec + I.S.uv_off[s] + (i - F.w);
}

// ---- factorization ---------------------------------------------------------------
// task (inst, s, j, -): zero column j of the front, then scatter the KKT slots
// of column j (j < w), eta added on the diagonal.
__global__ void __launch_bounds__(kBlock)
k_big_init(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred, double eta_force) {
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const double eta = pred == kPredAll ? eta_force : I.ctl->eta;
    const Front F = front_of(I, tk.y);
    const int j = tk.z;
    if (threadIdx.x == 0 && fwd_fused(I, tk.y, pred)) *fwd_entry(I, F, tk.y, j) = j < F.w ? I.rhs[I.perm[F.f + j]] : 0.0;
    for (int i = j + threadIdx.x; i < F.m; i += blockDim.x) *at(F, i, j) = 0.0;
    if (j >= F.w) return;
    __syncthreads();
    const int ld = F.m | 1;
    const int col = F.f + j;
    for (int t = I.kcol_ptr[col] + threadIdx.x; t < I.kcol_ptr[col + 1]; t += blockDim.x) {
        const int r = I.S.k_fpos[t] % ld;
        double v = I.kv[t];
        if (r == j) v += eta;
        F.L[r + (int64_t)j * F.m] = v;
    }
}

// task (inst, s, child position, child column jc): add column jc of the child's
// update block into the front through the child's relative row positions.
__global__ void __launch_bounds__(kBlock)
k_big_extend(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int c = I.S.child_list[I.S.child_ptr[tk.y] + tk.z];
    const int wc = I.S.sn_ptr[c + 1] - I.S.sn_ptr[c];
    const int nc = (int)(I.S.rows_ptr[c + 1] - I.S.rows_ptr[c]) - wc;
    const double* Uc = I.U + I.S.u_off[c];
    const int32_t* rel = I.S.rel + I.S.rel_off[c];
    const int jc = tk.w;
    const int rj = rel[jc];
    if (threadIdx.x == 0 && fwd_fused(I, tk.y, pred)) *fwd_entry(I, F, tk.y, rj) += I.uvec[I.S.uv_off[c] + jc];
    const auto* uc = global(Uc) + (int64_t)jc * nc;
    const auto* rg = global(rel);
    // kExtendDepth rows per thread at a time: their loads are issued together
    // (distinct rows of the child land on distinct entries of the front)
    for (int ic0 = jc + threadIdx.x; ic0 < nc; ic0 += kExtendDepth * kBlock) {
        int rr[kExtendDepth];
        double uv[kExtendDepth], tv[kExtendDepth];
#pragma unroll
        for (int u = 0; u < kExtendDepth; ++u) {
            const int ic = ic0 + u * kBlock;
            rr[u] = ic < nc ? rg[ic] : 0;
            uv[u] = ic < nc ? uc[ic] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kExtendDepth; ++u)
            tv[u] = ic0 + u * kBlock < nc ? *global(at(F, rr[u], rj)) : 0.0;
#pragma unroll
        for (int u = 0; u < kExtendDepth; ++u)
            if (ic0 + u * kBlock < nc) *global(at(F, rr[u], rj)) = tv[u] + uv[u];
    }
}

// task (inst, s, kb, -): factor the diagonal block D of columns [kb, kb + pw)
// in shared memory (panel-blocked, see partial_cholesky) and store it.  A pivot
// that is not positive and finite sets the instance's failure flag (eq. 12) and
// the arithmetic continues with pivot 1.
__global__ void __launch_bounds__(kBlock)
k_big_potrf(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    static_assert(kBigPanel == kWave, "diagonal blocks are staged as 64 x 64 triangles");
    __shared__ double D[kTri];
    __shared__ double fv[kBigPanel];   // the fused forward solve's entries of the panel
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int kb = tk.z;
    const int pw = min(kBigPanel, F.w - kb);
    constexpr int ldd = kBigPanel + 1;
    {
        double t[kStage];
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            const int e = threadIdx.x + s * kBlock, i = e % kBigPanel, j = e / kBigPanel;
            t[s] = (i < pw && j <= i) ? global(F.L)[(kb + i) + (int64_t)(kb + j) * F.m] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            const int e = threadIdx.x + s * kBlock;
            D[e % kBigPanel + (e / kBigPanel) * ldd] = t[s];
        }
    }
    const bool fw = fwd_fused(I, tk.y, pred);
    if (fw && (int)threadIdx.x < pw) fv[threadIdx.x] = *fwd_entry(I, F, tk.y, kb + threadIdx.x);
    __syncthreads();
    partial_cholesky<8>(D, SquareIdx{ldd}, pw, pw, &I.ctl->fail, fw ? fv : nullptr);
    for (int e = threadIdx.x; e < kBigPanel * kBigPanel; e += blockDim.x) {
        const int i = e % kBigPanel, j = e / kBigPanel;
        if (i < pw && j <= i) global(F.L)[(kb + i) + (int64_t)(kb + j) * F.m] = D[i + j * ldd];
    }
    if (fw && (int)threadIdx.x < pw) I.xp[F.f + kb + threadIdx.x] = fv[threadIdx.x];
}

// task (inst, s, kb, row block): solve x D^T = a for the rows
// [kb + pw + rb kRowBlock, ...) below the factored diagonal block D.  A full
// panel goes by blocks of 16 columns (blocked substitution): wave v holds its
// 16 rows in shared memory (leading dimension kLdx); for column block j the
// wave takes the block's 16 x 16 tile in the matrix-core layout (lane (li, lk)
// holds rows lk, lk + 4, lk + 8, lk + 12 of column li), subtracts the solved
// blocks' products with D's strict lower blocks on v_mfma_f64_16x16x4f64, then
// solves with D's 16 x 16 diagonal block column by column: the lanes of
// column k scale it by 1 / d_kk and the value reaches the later columns'
// lanes of its row by a shuffle.  A narrower last panel is solved in place,
// one lane per row.
constexpr int kLdx = 17;   // leading dimension of a wave's 16 rows in shared memory
__global__ void __launch_bounds__(kBlock)
k_big_trsm(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    __shared__ double D[kTri];   // strict lower triangle
    __shared__ double rd[kBigPanel];
    __shared__ double Xs[kBlock / kWave][kLdx * kBigPanel];
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int kb = tk.z;
    const int pw = min(kBigPanel, F.w - kb);
    constexpr int ldd = kBigPanel + 1;
    const int tid = threadIdx.x;
    const int r0 = kb + pw + tk.w * kRowBlock;
    if (r0 >= F.m) return;
    {
        double t[kStage];
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            const int e = tid + s * kBlock, i = e % kBigPanel, j = e / kBigPanel;
            t[s] = (i < pw && j <= i) ? global(F.L)[(kb + i) + (int64_t)(kb + j) * F.m] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            const int e = tid + s * kBlock, i = e % kBigPanel, j = e / kBigPanel;
            D[i + j * ldd] = i == j ? 0.0 : t[s];
            if (i == j) rd[i] = i < pw ? 1.0 / t[s] : 1.0;
        }
    }
    __syncthreads();
    const bool fw = fwd_fused(I, tk.y, pred);
    if (pw == kBigPanel) {
        static_assert(kRowBlock == 16 * (kBlock / kWave), "a wave takes 16 rows of the block");
        const int lane = tid & (kWave - 1), wv = tid / kWave, li = lane & 15, lk = lane >> 4;
        const int rw = r0 + 16 * wv;
        if (rw >= F.m) return;   // the whole wave (no barrier follows)
        double* X = Xs[wv];
        {
            double t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int col = 4 * u + lk, r = rw + li;
                t[u] = r < F.m ? global(F.L)[r + (int64_t)(kb + col) * F.m] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) X[li + (4 * u + lk) * kLdx] = t[u];
        }
        __builtin_amdgcn_wave_barrier();   // the wave's own shared-memory rows: program order suffices
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f64x4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = X[(4 * r + lk) + (16 * j + li) * kLdx];
#pragma unroll
            for (int i = 0; i < j; ++i)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double av = -X[li + (16 * i + 4 * s + lk) * kLdx];
                    const double bv = D[(16 * j + li) + (16 * i + 4 * s + lk) * ldd];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double rdk = rd[16 * j + k];
                const double dkl = D[(16 * j + li) + (16 * j + k) * ldd];   // zero unless li > k
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double own = li == k ? acc[r] * rdk : acc[r];
                    const double xk = __shfl(own, (lane & ~15) | k, kWave);
                    acc[r] = li > k ? fma(-xk, dkl, own) : own;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) X[(4 * r + lk) + (16 * j + li) * kLdx] = acc[r];
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int col = 4 * u + lk, r = rw + li;
            if (r < F.m) global(F.L)[r + (int64_t)(kb + col) * F.m] = X[li + col * kLdx];
        }
        if (fw) {   // each row takes the panel's product with its solution: lane (li, lk) sums 16 columns
            const double* xs = I.xp + F.f + kb + 16 * lk;
            double dot = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) dot = fma(X[li + (16 * lk + c) * kLdx], xs[c], dot);
            dot += __shfl_xor(dot, 16, kWave);
            dot += __shfl_xor(dot, 32, kWave);
            if (lk == 0 && rw + li < F.m) *fwd_entry(I, F, tk.y, rw + li) -= dot;
        }
    } else if (tid < kRowBlock) {
        // the last, narrower panel of a supernode: in place, one lane per row;
        // D's diagonal was zeroed, its reciprocal is in rd
        const int r = r0 + tid;
        if (r >= F.m) return;
        gdouble* row = global(F.L) + r + (int64_t)kb * F.m;
        const double* xs = I.xp + F.f + kb;
        double dot = 0.0;
        for (int k = 0; k < pw; ++k) {
            double acc = row[(int64_t)k * F.m];
            for (int j = 0; j < k; ++j) acc = fma(-row[(int64_t)j * F.m], D[k + j * ldd], acc);
            const double lk = acc * rd[k];
            row[(int64_t)k * F.m] = lk;
            if (fw) dot = fma(lk, xs[k], dot);
        }
        if (fw) *fwd_entry(I, F, tk.y, r) -= dot;
    }
}

// Tiles of one launch are handed out XCD by XCD: workgroups are dealt to the 8
// XCDs round-robin, so tile b % 8 * (n / 8) + b / 8 keeps neighbouring tiles
// (which share panel rows) on one XCD and its L2.
__device__ inline int xcd_tile(int b, int n) {
    const int full = (n / 8) * 8;
    return b < full ? (b % 8) * (n / 8) + b / 8 : b;
}

// C -= A B^T on one 64 x 64 tile, A and B the panel columns [k0, k0 + kw) of
// the tile's rows and columns.  Outer (Inner = false), task (inst, s, kb, tile):
// the lower triangle of the trailing block from kb + kw, kw = min(kBigOuter,
// w - kb).  Inner, task (inst, s, ki, tile): the rest of ki's outer panel,
// rows from ki + kw to m, columns [ki + kw, outer panel end), kw =
// min(kBigPanel, w - ki).  Wave v computes the 32 x 32 quarter (v / 2, v % 2).
template <bool Inner>
__global__ void __launch_bounds__(kBlock)
k_big_update(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    const int4 tk = tasks[xcd_tile(blockIdx.x, gridDim.x)];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int k0 = tk.z;
    const int kw = min(Inner ? kBigPanel : kBigOuter, F.w - k0);
    const int t0 = k0 + kw;
    int ti, tj;
    if (Inner) {
        const int cend = min(F.w, k0 - k0 % kBigOuter + kBigOuter);
        const int tc = (cend - t0 + kTile - 1) / kTile;
        ti = tk.w / tc;
        tj = tk.w - ti * tc;
    } else {
        ti = (int)((sqrt(8.0 * tk.w + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= tk.w) ++ti;
        while (ti * (ti + 1) / 2 > tk.w) --ti;
        tj = tk.w - ti * (ti + 1) / 2;
    }
    const int cmax = Inner ? min(F.w, k0 - k0 % kBigOuter + kBigOuter) : F.m;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int li = lane & 15, lk = lane >> 4;
    const int i0 = t0 + kTile * ti + 32 * (wv >> 1);
    const int j0 = t0 + kTile * tj + 32 * (wv & 1);
    if (j0 >= cmax || i0 >= F.m || j0 > i0 + 31) return;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // kUpdateDepth steps of 4 columns are loaded before their products, so the
    // loads of a step overlap one another instead of each waiting in turn
    // (columns past kw load zeros and add nothing)
    const gdouble* Lg = global(F.L);
    bool rok[2], cok[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) rok[a] = i0 + 16 * a + li < F.m;
#pragma unroll
    for (int b = 0; b < 2; ++b) cok[b] = j0 + 16 * b + li < cmax;
    for (int k4 = 0; k4 < kw; k4 += 4 * kUpdateDepth) {
        double av[kUpdateDepth][2], bv[kUpdateDepth][2];
#pragma unroll
        for (int u = 0; u < kUpdateDepth; ++u) {
            const int kk = k4 + 4 * u + lk;
            const gdouble* col = Lg + (int64_t)(k0 + kk) * F.m;
#pragma unroll
            for (int a = 0; a < 2; ++a) av[u][a] = (kk < kw && rok[a]) ? col[i0 + 16 * a + li] : 0.0;
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[u][b] = (kk < kw && cok[b]) ? col[j0 + 16 * b + li] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUpdateDepth; ++u)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][a], bv[u][b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * a + 4 * r + lk, j = j0 + 16 * b + li;
                if (i < F.m && j <= i && j < cmax) *global(at(F, i, j)) -= acc[a][b][r];
            }
}

// ---- solves ------------------------------------------------------------------------
// The columns of a large supernode are solved kChunk at a time.  Forward: one
// workgroup solves the chunk's triangle (the first chunk also gathers the
// right-hand side over the supernode's columns into xp and the rows below into
// its update vector, adding the children's update vectors), then the rows after
// the chunk (the rest of the diagonal part and the rows below) take the chunk's
// GEMV, split over workgroups.  Backward, from the last chunk: the rows below
// contribute L[w:m, k]^T x(rows below) to bsum (transposed GEMV), each chunk's
// triangle is solved by one workgroup, then the columns before the chunk take
// its transposed GEMV into bsum.  Sums over chunks run in a fixed order.
constexpr int kChunk = 256;

// Stage the lower triangle of the diagonal block [b0, b0 + bw)^2 of L in T
// (leading dimension kWave + 1) and the reciprocals of its diagonal in rd (1
// past bw); every load of a thread is issued before the first store.  The
// caller synchronizes.
__device__ inline void stage_triangle(const Front& F, int b0, int bw, double* T, double* rd) {
    double t[kStage];
#pragma unroll
    for (int s = 0; s < kStage; ++s) {
        const int e = threadIdx.x + s * kBlock, i = e % kWave, j = e / kWave;
        t[s] = (i < bw && j <= i) ? global(F.L)[(b0 + i) + (int64_t)(b0 + j) * F.m] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < kStage; ++s) {
        const int e = threadIdx.x + s * kBlock, i = e % kWave, j = e / kWave;
        if (j <= i) T[i + j * (kWave + 1)] = t[s];
        if (i == j) rd[i] = i < bw ? 1.0 / t[s] : 1.0;
    }
}

// Value of v in lane k of the wave, in every lane (k wave-uniform).
__device__ inline double lane_value(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

// forward, task (inst, s, chunk c): x[c0, c1) = L[c0:c1, c0:c1]^{-1} v[c0, c1)
// in xp, by blocks of 64 columns (the block's triangle staged in shared memory,
// wave 0 solves it, then the chunk's later rows take the block's update).
__global__ void __launch_bounds__(kBlock)
k_bigfwd_tri(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred, int which) {
    __shared__ double T[kTri];
    __shared__ double rd[kWave];
    __shared__ double v[kChunk];
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int s = tk.y, tid = threadIdx.x, nthr = blockDim.x;
    double* xs = I.xp + F.f;
    if (tk.z == 0) {
        const double* rhs = solve_in(I, which);
        double* us = I.uvec + I.S.uv_off[s];
        for (int k = tid; k < F.w; k += nthr) xs[k] = rhs[I.perm[F.f + k]];
        for (int i = tid; i < F.m - F.w; i += nthr) us[i] = 0.0;
        __syncthreads();
        for (int ci = I.S.child_ptr[s]; ci < I.S.child_ptr[s + 1]; ++ci) {
            const int c = I.S.child_list[ci];
            const int nc = (int)(I.S.uv_off[c + 1] - I.S.uv_off[c]);
            const double* uc = I.uvec + I.S.uv_off[c];
            const int32_t* rc = I.S.rel + I.S.rel_off[c];
            for (int i = tid; i < nc; i += nthr) {
                const int p = rc[i];
                if (p < F.w) xs[p] += uc[i];
                else us[p - F.w] += uc[i];
            }
            __syncthreads();
        }
    }
    const int c0 = tk.z * kChunk, cw = min(kChunk, F.w - c0);
    for (int k = tid; k < cw; k += nthr) v[k] = xs[c0 + k];
    for (int b0 = 0; b0 < cw; b0 += kWave) {
        const int bw = min(kWave, cw - b0), b1 = b0 + bw;
        stage_triangle(F, c0 + b0, bw, T, rd);
        __syncthreads();
        if (tid < kWave) {
            // lane j holds v_j; x_k leaves lane k through the scalar unit.  Lanes
            // j >= bw carry zeros (rd = 1 there, their entries of T are unused).
            const int j = tid;
            double vj = j < bw ? v[b0 + j] : 0.0;
#pragma unroll
            for (int k = 0; k < kWave; ++k) {
                const double xk = lane_value(vj, k) * rd[k];
                const double upd = fma(-T[j + k * (kWave + 1)], xk, vj);
                vj = j == k ? xk : (j > k && j < bw ? upd : vj);
            }
            if (j < bw) v[b0 + j] = vj;
        }
        __syncthreads();
        for (int i = b1 + tid; i < cw; i += nthr) {
            const gdouble* li = global(F.L) + (c0 + i) + (int64_t)(c0 + b0) * F.m;
            double acc = v[i];
            if (bw == kWave) {
#pragma unroll 32
                for (int k = 0; k < kWave; ++k) acc = fma(-li[(int64_t)k * F.m], v[b0 + k], acc);
            } else {
                for (int k = 0; k < bw; ++k) acc = fma(-li[(int64_t)k * F.m], v[b0 + k], acc);
            }
            v[i] = acc;
        }
        __syncthreads();
    }
    for (int k = tid; k < cw; k += nthr) xs[c0 + k] = v[k];
}

// forward, task (inst, s, chunk c, row block): rows i >= c1 of the block (one
// per thread): v[i] -= L[i, c0:c1) x[c0, c1), in xp (i < w) or in the update
// vector (i >= w).
__global__ void __launch_bounds__(kBlock)
k_bigfwd_gemv(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    __shared__ double x[kChunk];
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int c0 = tk.z * kChunk, cw = min(kChunk, F.w - c0), c1 = c0 + cw;
    for (int k = threadIdx.x; k < cw; k += blockDim.x) x[k] = I.xp[F.f + c0 + k];
    __syncthreads();
    const int i = c1 + tk.w * kSolveRows + threadIdx.x;
    if (i >= F.m) return;
    const gdouble* Li = global(F.L) + i + (int64_t)c0 * F.m;
    double acc = 0.0;
#pragma unroll 16
    for (int k = 0; k < cw; ++k) acc = fma(Li[(int64_t)k * F.m], x[k], acc);
    if (i < F.w) I.xp[F.f + i] -= acc;
    else I.uvec[I.S.uv_off[tk.y] + (i - F.w)] -= acc;
}

// backward, task (inst, s, column block): bsum[f + k] = L[w:m, k]^T x(rows below)
// for the block's columns; wave v takes columns k0 + v, k0 + v + 4, ..., lanes
// walk the rows (a butterfly sums the lanes).
__global__ void __launch_bounds__(kBlock)
k_bigbwd_below(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int32_t* rows = I.S.rows + I.S.rows_ptr[tk.y];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int k0 = tk.z * kSolveCols;
    for (int k = k0 + wv; k < min(F.w, k0 + kSolveCols); k += nw) {
        double acc = 0.0;
#pragma unroll 4
        for (int i = F.w + lane; i < F.m; i += kWave) acc = fma(global(F.L)[i + (int64_t)k * F.m], global(I.xp)[rows[i]], acc);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) I.bsum[F.f + k] = acc;
    }
}

// Whether bsum of a chunk's columns holds contributions: rows below the
// supernode, or a later chunk.
__device__ inline bool bsum_live(const Front& F, int c) { return F.m > F.w || (c + 1) * kChunk < F.w; }

// backward, task (inst, s, chunk c): v = xp[c0, c1) - bsum; solve
// L[c0:c1, c0:c1]^T x = v by blocks of 64 from the last (the block's triangle
// staged in shared memory, wave 0 solves it, then the chunk's earlier columns
// take the block's rows of L); writes xp and the unpermuted solution.
__global__ void __launch_bounds__(kBlock)
k_bigbwd_tri(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred, int which) {
    __shared__ double T[kTri];
    __shared__ double rd[kWave];
    __shared__ double v[kChunk];
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int c0 = tk.z * kChunk, cw = min(kChunk, F.w - c0);
    const bool live = bsum_live(F, tk.z);
    for (int k = tid; k < cw; k += nthr) v[k] = I.xp[F.f + c0 + k] - (live ? I.bsum[F.f + c0 + k] : 0.0);
    const int nblk = (cw + kWave - 1) / kWave;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int b0 = bi * kWave, bw = min(kWave, cw - b0);
        stage_triangle(F, c0 + b0, bw, T, rd);
        __syncthreads();
        if (tid < kWave) {
            // lane j holds v_j; rows k >= bw are skipped (x_k of a zero lane is 0)
            const int j = tid;
            double vj = j < bw ? v[b0 + j] : 0.0;
#pragma unroll
            for (int k = kWave - 1; k >= 0; --k) {
                const double xk = lane_value(vj, k) * rd[k];
                const double upd = fma(-T[k + j * (kWave + 1)], xk, vj);
                vj = j == k ? xk : (j < k && k < bw ? upd : vj);
            }
            if (j < bw) v[b0 + j] = vj;
        }
        __syncthreads();
        for (int c = tid; c < b0; c += nthr) {
            double acc = v[c];
            const gdouble* lc = global(F.L) + (int64_t)(c0 + c) * F.m + c0 + b0;
            if (bw == kWave) {
#pragma unroll 32
                for (int i = 0; i < kWave; ++i) acc = fma(-lc[i], v[b0 + i], acc);
            } else {
                for (int i = 0; i < bw; ++i) acc = fma(-lc[i], v[b0 + i], acc);
            }
            v[c] = acc;
        }
        __syncthreads();
    }
    double* out = solve_out(I, which);
    for (int k = tid; k < cw; k += nthr) {
        I.xp[F.f + c0 + k] = v[k];
        out[I.perm[F.f + c0 + k]] = v[k];
    }
}

// backward, task (inst, s, chunk c, column block): for the block's columns
// k < c0, bsum[f + k] (+)= L[c0:c1, k]^T x[c0, c1) (the first contribution of a
// supernode without rows below sets it); wave per column, lanes over the rows.
__global__ void __launch_bounds__(kBlock)
k_bigbwd_gemvt(const InstPtrs* __restrict__ Ia, const int4* __restrict__ tasks, int pred) {
    __shared__ double x[kChunk];
    const int4 tk = tasks[blockIdx.x];
    const InstPtrs& I = Ia[tk.x];
    if (!ctl_active(I.ctl, pred)) return;
    const Front F = front_of(I, tk.y);
    const int c0 = tk.z * kChunk, cw = min(kChunk, F.w - c0);
    for (int k = threadIdx.x; k < cw; k += blockDim.x) x[k] = I.xp[F.f + c0 + k];
    __syncthreads();
    const bool live = bsum_live(F, tk.z);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const int k0 = tk.w * kSolveCols;
    for (int k = k0 + wv; k < min(c0, k0 + kSolveCols); k += nw) {
        const gdouble* lk = global(F.L) + (int64_t)k * F.m + c0;
        double acc = 0.0;
        for (int i = lane; i < cw; i += kWave) acc = fma(lk[i], x[i], acc);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
        if (lane == 0) I.bsum[F.f + k] = (live ? I.bsum[F.f + k] : 0.0) + acc;
    }
}

}  // namespace

int big_row_block() { return kRowBlock; }
int big_tile() { return kTile; }
int big_solve_rows() { return kSolveRows; }
int big_solve_cols() { return kSolveCols; }
int big_chunk() { return kChunk; }

void launch_big(int kind, int pred, double eta_force, int which, const InstPtrs* I, const int4* tasks, int count,
                size_t lds_bytes, hipStream_t st) {
    if (count <= 0) return;
    switch (kind) {
        case kBigInit:
            hipLaunchKernelGGL(k_big_init, dim3(count), dim3(kBlock), 0, st, I, tasks, pred, eta_force);
            break;
        case kBigExtend:
            hipLaunchKernelGGL(k_big_extend, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigPotrf:
            hipLaunchKernelGGL(k_big_potrf, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigTrsm:
            hipLaunchKernelGGL(k_big_trsm, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigUpdate:
            hipLaunchKernelGGL(k_big_update<false>, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigUpdateInner:
            hipLaunchKernelGGL(k_big_update<true>, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigFwdTri:
            hipLaunchKernelGGL(k_bigfwd_tri, dim3(count), dim3(kBlock), 0, st, I, tasks, pred, which);
            break;
        case kBigFwdGemv:
            hipLaunchKernelGGL(k_bigfwd_gemv, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigBwdBelow:
            hipLaunchKernelGGL(k_bigbwd_below, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        case kBigBwdTri:
            hipLaunchKernelGGL(k_bigbwd_tri, dim3(count), dim3(kBlock), 0, st, I, tasks, pred, which);
            break;
        case kBigBwdGemvT:
            hipLaunchKernelGGL(k_bigbwd_gemvt, dim3(count), dim3(kBlock), 0, st, I, tasks, pred);
            break;
        default:
            break;
    }
}

}  // namespace nmpc
