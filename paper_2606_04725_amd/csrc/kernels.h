// Device-side structures and launch wrappers shared by the HIP translation
// units.  Every kernel works on a batch of instances (a single solve is a
// batch of one): per-instance pointers live in an InstPtrs array and the
// per-instance interior-point decisions in a Ctl block, both in device memory,
// so that a pass of the method needs no host decision and can be captured as a
// graph.  Each kernel file exposes plain host launch functions so no kernel
// symbol crosses a translation unit.
#ifndef NMPC_KERNELS_H
#define NMPC_KERNELS_H

#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/nmpc.h"
#include "distill_layout.h"
#include "plate_layout.h"
#include "reflux_layout.h"

namespace nmpc {

constexpr int kBlock = 256;          // threads per block of every vector kernel
constexpr int kFactorBlock = 256;    // threads per supernode group
constexpr int kPanel = 8;            // pivot columns per blocked step of a front
constexpr int kMediumFront = 256;    // largest front one workgroup factors in a global buffer
constexpr int kMaxQ = 12;            // reduced quantities per phase
constexpr int kMaxSeed = 16;         // controls per stage the sensitivity seed can hold
constexpr int kFilterCapMax = 256;   // filter entries an instance can hold

struct DistillConst {
    double dt, alpha, F, rho;
};

// Stage-model family: constants its generated kernels read.  tag names the
// kernels meant for the instance; pc is null when the state rows hold the
// previous states with coefficient -1 each (implicit Euler), else the nx x nx
// coefficient matrix (row-major) of the previous states in the state rows.
struct StageConst {
    double dt;
    unsigned long long tag;
    const double* pc;
    double* scratch;   // H x (the model's per-stage scratch) doubles, or null
};

// Per-supernode read-only symbolic data of one instance.
// What the extend-add of the child at one position of child_list reads:
// its update block (u_off), its rows' positions in the parent (rel_off), its
// update vector (uv_off) and its number of rows below its columns (nc).
struct ChildRec {
    int64_t u_off, rel_off, uv_off;
    int32_t nc, child;
};

struct SnView {
    const int32_t* sn_ptr;
    const int64_t* rows_ptr;
    const int32_t* rows;
    const int32_t* child_ptr;
    const int32_t* child_list;
    const ChildRec* child_rec;    // per child_list position
    const ChildRec* first_recs;   // per supernode: the records of its first two children (zero past the last)
    const int64_t* l_off;
    const int64_t* u_off;
    const int64_t* uv_off;
    const int64_t* rel_off;
    const int32_t* rel;
    const int32_t* k_ptr;
    const int32_t* k_fpos;
    const int32_t* sched_nodes;   // supernodes in launch-schedule order
    const int32_t* fused;         // 1: the Newton step's forward solve runs inside the factor kernel
};

// Phases of one Newton iteration of Algorithm 2 for one instance:
//   A  evaluate, optimality errors, convergence test, barrier update
//   B  condensed assembly (eqs. 14, 17), then the first factorization (eta = 0)
//   F  factorization retried with a larger eta (inertia correction)
//   S  solves (eqs. 22-25), remaining directions, fraction to the boundary (eq. 26)
//   T  one trial point of the backtracking line search
//   C  one second-order correction of the first trial point
//   U  accepted step: update, next iteration
enum Phase : int { kPhA = 0, kPhB = 1, kPhF = 2, kPhS = 3, kPhT = 4, kPhC = 5, kPhU = 6, kPhDone = 7 };
// predicate values of the launch wrappers: a phase, or one of these
constexpr int kPredAll = -1;       // every instance, whatever its phase
constexpr int kPredFactor = 100;   // phases B and F

constexpr int kStatusRunning = -1;

// Interior-point state of one instance, read and written on the device.
struct Ctl {
    double mu, tau, alpha, eta, eta_last, f, E0, gamma;
    // filter line search: violation and barrier objective at the iterate, the
    // directional derivative of phi, the minimal step, the theta bounds and the
    // barrier value the filter belongs to
    double theta, phi0, dphi, amin, theta_max, theta_min, filter_mu;
    // second-order corrections: first trial step, last correction's step and violation
    double alpha0, soc_a, soc_theta;
    // l1-merit fallback: first step of the search, max |omega + d_omega| of the
    // direction, the penalty (kept over the solve)
    double amax0, om_max, nu;
    int ls_merit;        // the current search runs on the l1 merit
    int merit_trials;    // trial points of the merit search
    int filter_n;        // entries in the instance's filter
    int soc_p;           // corrections done in the current line search
    int use_soc;         // the accepted step is the correction's
    int status;          // kStatusRunning or a final nmpc status
    int phase;
    int it;              // accepted Newton steps
    int fail;            // set by the factorization: a pivot is not positive and finite
    int trials;          // trial points of the current line search
    int factorizations, ls_trials;
    // HyKKT (equalities kept exact, Newton system by the Cholesky factor of
    // K_gamma = K_c + hk_gamma J_c^T J_c and conjugate gradients on the Schur
    // complement): mode flag, and the running CG of the current step
    int hyk;
    int cg_it, cg_done, cg_total;
    double hk_gamma, cg_rr, cg_stop, cg_alpha, cg_beta;
};

__host__ __device__ inline bool ctl_active(const Ctl* c, int pred) {
    if (pred == kPredAll) return true;
    const int ph = c->phase;
    if (pred == kPredFactor) return ph == kPhB || ph == kPhF;
    return ph == pred;
}

// Loads through a pointer in the global address space are global (not flat)
// instructions: they count only against the vector-memory counter, so waits
// for shared memory do not also wait for them.
typedef __attribute__((address_space(1))) double gdouble;
template <class T>
__device__ inline const __attribute__((address_space(1))) T* global(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Everything a kernel needs to know about one instance.
struct InstPtrs {
    int family;
    int n, mc, md, ml, m, nx, nu, H;
    int64_t nnzk;
    DistillDims dd;
    DistillConst dc;
    PlateDims pd;
    PlateConst pc;
    RefluxDims rd;
    RefluxConst rc;
    StageConst gm;
    int ns, rps;        // variables and (dynamics block) equality rows per stage
    int nsp, ntr;       // setpoint and disturbance-trajectory lengths of the family
    // structure
    const int32_t *jptr, *jcol, *jt_ptr, *jt_slot, *jt_row;
    const double *lb, *ub;
    const int32_t* perm;
    SnView S;
    const int32_t *k_wslot, *k_diag, *kc_ptr, *kc_a, *kc_b, *kc_r;
    // parameters
    const double *x0, *zF, *uprev, *setp;
    // iterate and work vectors
    double *y, *s, *om, *be, *zl, *zu;
    double *c, *d, *jv, *wv, *grad, *fterm, *gtw, *sig, *rhs, *dy, *xp;
    double *Q, *r2, *r4, *qeff, *vcomb;
    double *ds, *dom, *dbe, *dzl, *dzu, *yt, *st;
    // second-order correction: r1 of the step, corrected residual and its
    // row combinations, right-hand side and directions
    double *r1v, *r4s, *vcomb_s, *rhs_s, *dy_s, *ds_s, *dom_s, *dbe_s, *dzl_s, *dzu_s;
    double *kv, *L, *U, *uvec;
    double *adj_rhs, *adj_w, *adj_out, *adj_b, *adj_d, *adj_lam, *adj_qr;
    double* adj_seed;   // seed of the sensitivities: u1 part (nu values), then the objective's
    const int32_t *wf_ptr, *wf_slot, *wf_col;   // Hessian rows, both triangles: (slot, column)
    double* gscratch;
    int64_t gstride;
    const int32_t* kcol_ptr;   // KKT slots of each permuted column: [kcol_ptr[j], kcol_ptr[j + 1])
    double* bsum;     // large-supernode backward solves: rows-below products per column
    double* part;     // reduction partials: kMaxQ rows of this instance's blocks
    double* filter;   // (theta, phi) pairs, kFilterCapMax of them
    // HyKKT: CG iterate, residual, direction and S-product over the equality
    // rows (m_c each); J_c^T p and its solve with the factor (n each)
    double *hk_x, *hk_r, *hk_p, *hk_sp, *hk_t, *hk_w;
    Ctl* ctl;
};

// Layout check between the library and the code objects of generated stage
// models (both read InstPtrs): the library refuses a code object whose
// nmpc_stage_abi differs.
constexpr unsigned int kStageAbiVersion = 2;
constexpr unsigned int kStageAbi = kStageAbiVersion * 100000u + (unsigned int)sizeof(InstPtrs);

// Right-hand side and solution of the solves: 0 rhs -> dy (Newton step),
// 1 yt -> dzl (single-solve entry point), 2 adj_rhs -> adj_w (sensitivities),
// 3 adj_rhs -> adj_d (refinement corrections of the sensitivities),
// 4 rhs_s -> dy_s (second-order correction), 5 hk_t -> hk_w (HyKKT products
// with K_gamma^{-1}).
__host__ __device__ inline const double* solve_in(const InstPtrs& I, int which) {
    return which == 0 ? I.rhs : (which == 1 ? I.yt : (which == 4 ? I.rhs_s : (which == 5 ? I.hk_t : I.adj_rhs)));
}
__host__ __device__ inline double* solve_out(const InstPtrs& I, int which) {
    return which == 0 ? I.dy
                      : (which == 1 ? I.dzl
                                    : (which == 2 ? I.adj_w : (which == 3 ? I.adj_d : (which == 5 ? I.hk_w : I.dy_s))));
}

// Block -> instance map of one index space.  Instance i owns blocks
// [bfirst[i], bfirst[i + 1]); binst[b] is the instance of block b.
struct Space {
    const int32_t* binst;
    const int32_t* bfirst;
    int blocks;
};
enum SpaceKind : int { kSpN = 0, kSpNML = 1, kSpM = 2, kSpK = 3, kSpMN = 4, kSpMax = 5, kNumSpaces = 6 };
// size of an instance in each space
__host__ __device__ inline int64_t space_size(const InstPtrs& I, int kind) {
    switch (kind) {
        case kSpN: return I.n;
        case kSpNML: return (int64_t)I.n + I.ml;
        case kSpM: return I.m;
        case kSpK: return I.nnzk;
        case kSpMN: return (int64_t)I.m + I.n;
        default: return I.n > I.ml ? I.n : I.ml;
    }
}

// Instance of the calling block and the block's index within that instance.
__device__ inline int block_inst(const Space& sp, int& local_block) {
    const int i = sp.binst[blockIdx.x];
    local_block = (int)blockIdx.x - sp.bfirst[i];
    return i;
}

// Interior-point constants the device decisions use.
struct DevOpts {
    double tol, mu_min, kappa_eps, kappa_mu, theta_mu, tau_min, armijo, kappa_sigma;
    double eta_first, eta_min, eta_max, kp_first, kp, km;
    double g_theta, g_phi, s_theta, s_phi, delta, amin_frac, theta_max_fact, theta_min_fact, soc_kappa;
    int ls_max, max_iter, filter_cap, soc_max, merit_fallback, fixed_mu;
    double cg_tol;
    int cg_max;
};

// One group of supernodes of one instance: sched_nodes[begin .. end), walked in
// order by one workgroup; slot selects the workgroup's global front buffer.
struct Group {
    int inst, begin, end, slot;
};

// ---- model evaluation (kernels_model.hip) -------------------------------------------
// Source of the point and multipliers: the iterate (y, om), the trial point
// (yt; values only), or a caller-given point staged in (yt, dom).
enum EvalSrc : int { kSrcIter = 0, kSrcTrial = 1, kSrcUser = 2 };
// full: c, d, Jacobian values, Lagrangian Hessian values, gradient and objective
// terms; otherwise c, d and objective terms.  Space kSpN, one lane per variable.
void launch_eval_distill(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st);
void launch_eval_plate(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st);
void launch_eval_reflux(bool full, int src, int pred, const InstPtrs* I, const Space& sp, hipStream_t st);

// ---- interior-point vector kernels and decisions (kernels_ipm.hip) ----------------
struct IpmSpaces {
    Space sp[kNumSpaces];
};
void launch_phaseA(const InstPtrs* I, const IpmSpaces& S, int ninst, int pred, const DevOpts& o, bool decide,
                   hipStream_t st);
void launch_assemble(const InstPtrs* I, const IpmSpaces& S, int pred, hipStream_t st);
void launch_decideF(const InstPtrs* I, int ninst, const DevOpts& o, hipStream_t st);
void launch_phaseE(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st);
void launch_trial(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
void launch_phaseT(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st);
// second-order correction, before its solve (rows, right-hand side) and after
// it (directions and step bound, trial point), then its acceptance test
void launch_soc_prepare(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
void launch_soc_step(const InstPtrs* I, const IpmSpaces& S, int ninst, hipStream_t st);
void launch_soc_decide(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, hipStream_t st);
// update of the accepted instances, then close the pass: running count -> *running
void launch_update(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* running,
                   hipStream_t st);
void launch_cold_start(const InstPtrs* I, const IpmSpaces& S, double bound_push, double slack_push, double mu0,
                       bool after_eval, hipStream_t st);
// HyKKT step (instances in phase S with the HyKKT flag): CG start after the
// solve of the right-hand side, one CG iteration as J_c^T p (pre), the solve
// hk_t -> hk_w that the caller enqueues, and the rest of the iteration (post);
// both write the number of instances whose CG still runs to *count.  finish:
// the right-hand side of the final solve.  from_lifted: convert the held
// Lifted-KKT iterate.
void launch_hk_cg_start(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* count,
                        hipStream_t st);
void launch_hk_cg_pre(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
void launch_hk_cg_post(const InstPtrs* I, const IpmSpaces& S, int ninst, const DevOpts& o, int* count,
                       hipStream_t st);
void launch_hk_finish(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
void launch_hk_from_lifted(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
// shifted warm start: every stage-indexed quantity of the held iterate moves
// one stage earlier, the last stage keeps its own
void launch_shift(const InstPtrs* I, const IpmSpaces& S, hipStream_t st);
void launch_set_fail(const InstPtrs* I, int ninst, int value, hipStream_t st);
// sensitivities: rhs = seed_obj grad f + S_u^T seed_u, and the parameter contractions
void launch_adj_seed(const InstPtrs* I, const Space& spN, hipStream_t st);   // seed from adj_seed
void launch_cold_guess(const InstPtrs* I, const Space& spN, hipStream_t st);
// lam = omega+ - omega- and the inequality multipliers of instance 0 into caller buffers (NULL skips)
void launch_export_duals(const InstPtrs* I, double* lam, double* om_d, int rows, hipStream_t st);
// out = [x0 (nx) | setpoint (nsp) | trajectory (ntr) | u_prev (nu)] for instance 0
void launch_adj_gather(const InstPtrs* I, int family, int nx, hipStream_t st);
void launch_x0_map(const double* lam, int64_t stride, const double* pc, double* out, int nx, int K, hipStream_t st);
// Refinement of w = K^{-1} b against the uncondensed system [K0 J^T; J -Q^{-1}]
// (K0 = W + Sigma + eta I): start sets lam = Q J w; residual forms
// adj_rhs = b - K0 w - J^T lam + J^T qr with qr = lam - Q J w; update adds the
// correction adj_d: w += d, lam += Q J d - qr.
void launch_adj_refine(int step, const InstPtrs* I, const IpmSpaces& S, double eta, hipStream_t st);

// ---- numeric factorization and solves (kernels_linalg.hip) -------------------------
// Multifrontal Cholesky (eqs. 20-21) of a list of groups, one workgroup per
// group, for instances matching pred (kPredFactor during a solve) with eta
// from the control block, or every instance with eta_force (pred kPredAll).
// lds: fronts in shared memory (lds_bytes), else in the instance's gscratch.
// variant: (threads per workgroup, panel width) = 0 (256, 8), 1 (512, 8),
// 2 (128, 8), 3 (256, 4), 4 (512, 4); the same arithmetic up to the panel width.
constexpr int kFactorVariants = 5;
void launch_factor_groups(bool lds, int variant, int pred, double eta_force, const InstPtrs* I, const Group* g,
                          int groups, size_t lds_bytes, hipStream_t st);
// Forward (eq. 23, rhs permutation fused) and back (eqs. 24-25, inverse
// permutation fused) substitution over groups, vectors chosen by which.
void launch_fwd_groups(int pred, int which, const InstPtrs* I, const Group* g, int groups, size_t lds_bytes,
                       hipStream_t st);
void launch_bwd_groups(int pred, int which, const InstPtrs* I, const Group* g, int groups, size_t lds_bytes,
                       hipStream_t st);
// Raise the dynamic shared-memory limit of the front kernels (once per process).
hipError_t linalg_configure(size_t max_lds_bytes);

// ---- large supernodes (kernels_big.hip) ---------------------------------------------
constexpr int kBigPanel = 64;   // pivot columns per panel step of a large front
constexpr int kBigOuter = 512;  // columns per outer panel (one trailing update each)
enum BigKind : int {
    kBigInit = 1,       // task (inst, s, column, -)
    kBigExtend = 2,     // task (inst, s, child position, child column)
    kBigPotrf = 3,      // task (inst, s, kb, -)
    kBigTrsm = 4,       // task (inst, s, kb, row block)
    kBigUpdate = 5,     // task (inst, s, kb, lower-triangle tile)
    kBigFwdTri = 6,     // task (inst, s, chunk, -)
    kBigFwdGemv = 7,    // task (inst, s, chunk, row block)
    kBigBwdBelow = 8,   // task (inst, s, column block, -)
    kBigBwdTri = 9,     // task (inst, s, chunk, -)
    kBigUpdateInner = 10,  // task (inst, s, ki, rectangular tile)
    kBigBwdGemvT = 11   // task (inst, s, chunk, column block)
};
// One step for every task of a list (predicate and eta as for the groups;
// which selects the solve vectors).
void launch_big(int kind, int pred, double eta_force, int which, const InstPtrs* I, const int4* tasks, int count,
                size_t lds_bytes, hipStream_t st);
int big_row_block();
int big_tile();
int big_solve_rows();
int big_solve_cols();
int big_chunk();   // columns per chunk of a large supernode's solves

}  // namespace nmpc

#endif
