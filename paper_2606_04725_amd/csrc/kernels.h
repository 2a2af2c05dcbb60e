// Launch wrappers shared by the device translation units.  Each kernel file
// exposes plain host functions so no kernel symbol crosses a translation unit.
#ifndef NMPC_KERNELS_H
#define NMPC_KERNELS_H

#include <hip/hip_runtime.h>
#include <cstdint>

#include "distill_layout.h"

namespace nmpc {

constexpr int kBlock = 256;          // threads per block of every vector kernel
constexpr int kFactorBlock = 256;    // threads per supernode front
constexpr int kPanel = 8;            // pivot columns per blocked step of a front
constexpr int kRelInts = 512;        // shared-memory ints reserved ahead of a front (relative positions)

struct DistillConst {
    double dt, alpha, F, rho, xD, xB;
};

// Per-supernode read-only symbolic data on the device.
struct SnView {
    const int32_t* sn_ptr;
    const int64_t* rows_ptr;
    const int32_t* rows;
    const int32_t* child_ptr;
    const int32_t* child_list;
    const int64_t* l_off;
    const int64_t* u_off;
    const int64_t* uv_off;
    const int64_t* rel_off;
    const int32_t* rel;
    const int32_t* k_ptr;
    const int32_t* k_fpos;
};

// Model evaluation (Section 4.1 family), one thread per (stage, variable).
// full = true: c, d, Jacobian, Hessian of the Lagrangian (multipliers from om),
// gradient and objective terms; full = false: c, d and objective terms only.
void launch_eval_distill(bool full, const DistillDims& D, const DistillConst& C, const double* y,
                         const double* x0, const double* zF, const double* uprev, const double* om,
                         const int32_t* jptr, int mc, double* c, double* d, double* jv, double* wv,
                         double* grad, double* fterm, hipStream_t st);

// Numeric multifrontal Cholesky (eqs. 20-21) of a list of supernode groups:
// workgroup b factors nodes[gptr[b] .. gptr[b+1]) in order.  lds: every front
// fits in shared memory (bytes = lds_bytes), otherwise fronts live in gscratch.
void launch_factor_groups(bool lds, const int32_t* nodes, const int32_t* gptr, int groups, size_t lds_bytes,
                          const SnView& S, const double* kv, double eta, double* L, double* U, int* fail,
                          double* gscratch, int64_t gstride, hipStream_t st);
// Forward substitution (eq. 23) over groups, permutation of the rhs fused;
// lds_bytes holds one front-length vector.
void launch_fwd_groups(const int32_t* nodes, const int32_t* gptr, int groups, size_t lds_bytes, const SnView& S,
                       const double* L, double* uvec, const double* rhs, const int32_t* perm, double* xp,
                       hipStream_t st);
// Back substitution (eqs. 24-25) over groups, inverse permutation fused.
void launch_bwd_groups(const int32_t* nodes, const int32_t* gptr, int groups, size_t lds_bytes, const SnView& S,
                       const double* L, double* xp, const int32_t* perm, double* out, hipStream_t st);
// Raise the dynamic shared-memory limit of the front kernels (once per process).
hipError_t linalg_configure(size_t max_lds_bytes);

}  // namespace nmpc

#endif
