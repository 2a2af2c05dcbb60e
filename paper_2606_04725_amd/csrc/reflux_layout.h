// Slot layout of the reflux-ratio column of the paper's distillation case
// study (Section 4.1, its OCP as written there).
//
// N trays (tray 1 the condenser, tray N the reboiler), feed tray Nf.
// Variables are stage-major, ns = 2 N + 4 per stage:
//   [x_1 .. x_N, u, y_1 .. y_N, L, V, S]   (local indices 0..N-1, N, N+1..2N, 2N+1, 2N+2, 2N+3)
// Equality rows are stage-major, rps = 2 N + 3 per stage: tray i's implicit
// Euler residual (row i - 1), tray i's equilibrium y_i - phi(x_i) (row
// N + i - 1), then L - u D, V - L - D, S - L - F.  No inequality rows.
//
// Jacobian rows, columns ascending: a tray row holds x_{k-1,i} (k > 0), then
// of stage k: tray 1: x_1, y_2, V; trays 2..Nf-1: x_{i-1}, x_i, y_i, y_{i+1},
// L, V; tray Nf: the same plus S; trays Nf+1..N-1: x_{i-1}, x_i, y_i, y_{i+1},
// V, S; tray N: x_{N-1}, x_N, y_N, V, S.  Equilibrium row: x_i, y_i.  Flow
// rows: (u, L), (L, V), (L, S).
//
// Lower Hessian slots, 3 N per stage at k * 3 N:
//   [0, N)            (x_i, x_i)
//   N                 (u, u)
//   [N + 1, N + Nf)   (L, x_j), j = 1 .. Nf - 1
//   [N + Nf, 2 N)     (S, x_j), j = Nf .. N - 1
//   2 N               (V, x_1)
//   [2 N + 1, 3 N)    (V, y_j), j = 2 .. N
#ifndef NMPC_REFLUX_LAYOUT_H
#define NMPC_REFLUX_LAYOUT_H

#include <hip/hip_runtime.h>

struct RefluxDims {
    int N, Nf, ns, rps, H;
};

struct RefluxConst {
    double dt, alpha, F, D, xf, Ac, At, Ar, wu;
};

// nonzeros of the Jacobian row of tray i (1-based) at stage k
__host__ __device__ inline int rx_tray_nnz(const RefluxDims& D, int k, int i) {
    int c;
    if (i == 1) c = 3;
    else if (i < D.Nf) c = 6;
    else if (i == D.Nf) c = 7;
    else if (i < D.N) c = 6;
    else c = 5;
    return c + (k > 0 ? 1 : 0);
}

__host__ __device__ inline int rx_wstage(const RefluxDims& D) { return 3 * D.N; }

#endif
