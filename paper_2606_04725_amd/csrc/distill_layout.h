// Slot layout of the transcribed distillation-column OCP (Section 4.1 family).
//
// Variables are stage-major: stage k (0-based, k = 0..H-1 for stages 1..H)
// holds [x_0 .. x_{N+1}, R, V], ns = N + 4 entries, at k * ns.
// Equality rows c: row k * nx + i (nx = N + 2) is the implicit-Euler residual
// of state i at stage k.  With a control horizon (stages hc..H-1 held),
// equality rows H nx + 2 (k - hc) + j, k = hc..H-1, j = 0 (R) / 1 (V), are the
// holds u_{k,j} - u_{k-1,j} = 0 (two slots: u_{k-1,j} then u_{k,j}); hc = H
// without holds.  Inequality rows d: m_c + 2k (R - V <= 0) and
// m_c + 2k + 1 (V - R - F <= 0).
//
// Jacobian rows are stored CSR with columns ascending; row (k, i) holds, in
// order: x_{k-1,i} (k > 0), x_{k,i-1} (i > 0), x_{k,i}, x_{k,i+1} (i < nx-1),
// R_k (i > 0), V_k.  Each d row holds R_k, V_k.
//
// Lower Hessian slots: stage block k at k * (3 nx + 2):
//   [0, nx)             (x_i, x_i)
//   [nx, 2 nx)          (R, x_i)
//   2 nx                (R, R)
//   [2 nx + 1, 3 nx + 1) (V, x_i)
//   3 nx + 1            (V, V)
// followed, after all H blocks, by the cross-stage move-penalty pair for
// k = 1..H-1 at H (3 nx + 2) + 2 (k - 1): (R_k, R_{k-1}), (V_k, V_{k-1}).
#ifndef NMPC_DISTILL_LAYOUT_H
#define NMPC_DISTILL_LAYOUT_H

#include <hip/hip_runtime.h>

struct DistillDims {
    int N, nx, ns, H, fd;
    int hc;   // first held stage (0-based) of the control horizon; H: no holds
};

__host__ __device__ inline int dl_row_nnz(const DistillDims& D, int k, int i) {
    int nb = (i == 0 || i == D.nx - 1) ? 2 : 3;
    return (k > 0 ? 1 : 0) + nb + (i > 0 ? 1 : 0) + 1;
}

__host__ __device__ inline int dl_wstage(const DistillDims& D) { return 3 * D.nx + 2; }

__host__ __device__ inline int dl_wcross(const DistillDims& D, int k) {
    return D.H * dl_wstage(D) + 2 * (k - 1);
}

__host__ __device__ inline int dl_nnz_w(const DistillDims& D) {
    return D.H * dl_wstage(D) + 2 * (D.H - 1);
}

#endif
