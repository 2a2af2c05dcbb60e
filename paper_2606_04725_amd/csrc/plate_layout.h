// Slot layout of the transcribed heated-plate OCP (Section 4.2 family).
//
// Grid: G x G interior nodes, node p = b G + a.  Heater segment s = 4 e + j on
// edge e (0 bottom b = -1, 1 right a = G, 2 top b = G, 3 left a = -1) drives the
// ghost nodes with edge coordinate in [j q, (j + 1) q), q = G / 4.
//
// Variables are stage-major: stage k holds [T_0 .. T_{G^2 - 1}, u_0 .. u_15],
// ns = G^2 + 16 entries, at k * ns.  Equality row k * G^2 + p is the
// implicit-Euler residual of node p at stage k; there are no inequality rows.
//
// Jacobian row (k, p) holds, columns ascending: T_{k-1,p} (k > 0), T_{k,p-G}
// (b > 0), T_{k,p-1} (a > 0), T_{k,p}, T_{k,p+1} (a < G - 1), T_{k,p+G}
// (b < G - 1), then the controls of its ghost neighbours in increasing segment
// order (bottom, right, top, left).  The Lagrangian Hessian is diagonal: slot j
// is variable j.
#ifndef NMPC_PLATE_LAYOUT_H
#define NMPC_PLATE_LAYOUT_H

#include <hip/hip_runtime.h>

struct PlateDims {
    int G, nx, ns, H, q;
};

struct PlateConst {
    double dt, kap, inv_h2;   // kap: half the conductivity slope
};

__host__ __device__ inline int pl_row_nnz(const PlateDims& D, int k, int p) {
    const int b = p / D.G, a = p - b * D.G;
    int c = (k > 0) + 1 + (b > 0) + (a > 0) + (a < D.G - 1) + (b < D.G - 1);
    c += (b == 0) + (a == D.G - 1) + (b == D.G - 1) + (a == 0);
    return c;
}

#endif
