// Internal host-side data structures of the NMPC library.
#ifndef NMPC_INTERNAL_H
#define NMPC_INTERNAL_H

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nmpc.h"

namespace nmpc {

// Fixed structure of one transcribed OCP (eq. 6): sizes, sparsity patterns and
// bounds, built once on the host by the family's transcription.
struct Structure {
    nmpc_structure desc{};
    int n = 0, m_c = 0, m_d = 0, nx = 0, nu = 0, H = 0;
    // Jacobian of [c; d] in CSR (rows m_c + m_d), columns ascending per row
    std::vector<int32_t> jptr, jcol, jrow;
    // lower Hessian pattern, slot order as the eval kernel writes it
    std::vector<int32_t> wrow, wcol;
    std::vector<double> lb, ub;
    int64_t nnz_k = 0;
    // stage-model family: copies of the descriptor's data (desc.stage_model
    // is cleared: the caller's descriptor is not kept)
    struct StageModel {
        int ns = 0, rps = 0, nsp = 0, nw = 0, nwx = 0, nd = 0;
        bool traj = false;
        uint64_t tag = 0;
        std::vector<unsigned char> code;
        std::vector<double> pc;   // nx x nx coefficients of the previous states in the state rows, row-major
                                  // (left empty when they are minus the identity)
        bool pc_minus_identity = false;
        int64_t scratch = 0;      // per-stage scratch doubles of the kernels (then they have a reduce kernel)
    } gm;
};

// Result of SymCholesky (eqs. 18-19) plus every map the numeric phase needs.
struct Symbolic {
    int n = 0;
    std::vector<int32_t> perm, iperm, parent, colcount;
    int64_t nnz_l = 0, flops = 0;
    // supernodes
    int nsn = 0;
    std::vector<int32_t> sn_ptr;              // first column of each supernode (+ n)
    std::vector<int64_t> sn_rows_ptr;         // into sn_rows
    std::vector<int32_t> sn_rows;             // sorted rows, own columns first
    std::vector<int32_t> sn_parent;
    std::vector<int32_t> child_ptr, child_list;
    std::vector<int32_t> level_ptr, level_list;  // bottom-up levels of the supernodal tree
    int depth = 0;
    int max_front = 0;
    // storage offsets
    std::vector<int64_t> l_off;               // rows * width panel per supernode
    std::vector<int64_t> u_off;               // (rows - width)^2 update block per supernode, in a reused pool
    std::vector<int64_t> uv_off;              // (rows - width) update vector per supernode
    std::vector<int64_t> rel_off;             // relative positions of below rows in the parent
    std::vector<int32_t> rel;
    int64_t stored_l = 0, stored_u = 0, stored_uv = 0;
    // KKT slots in factor order (sorted by permuted column, then row)
    std::vector<int32_t> k_ptr;               // per supernode
    std::vector<int32_t> kcol_ptr;            // per permuted column
    std::vector<int32_t> k_fpos;              // position in the supernode front (r + c * (rows | 1): odd leading dimension)
    std::vector<int32_t> k_orow, k_ocol;      // original (row, col), row >= col
    std::vector<int32_t> k_wslot;             // Hessian slot or -1
    std::vector<int32_t> k_diag;              // variable index if diagonal else -1
    std::vector<int32_t> kc_ptr, kc_a, kc_b, kc_r;  // J^T Q J contributions per slot
    // transposed Jacobian: per variable, (slot, row)
    std::vector<int32_t> jt_ptr, jt_slot, jt_row;
};

constexpr int kFilterCapacity = 256;   // largest filter_cap an instance's filter storage holds

struct Device;   // device-side buffers, defined in the HIP translation unit
struct Batch;    // instances solved together, defined in the HIP translation unit

struct Problem {
    Structure st;
    Symbolic sym;
    bool analyzed = false;
    bool have_iterate = false;
    // the held iterate belongs to the parameters currently set (cleared by a
    // parameter change, set by a solve or an explicit iterate)
    bool params_current = false;
    // the held iterate is a HyKKT one (equality rows hold lambda, no slacks)
    bool iter_hyk = false;
    int64_t solution_id = 0;   // increases with every iterate the handle takes
    // parameters (host copies)
    std::vector<double> x0, setpoint, traj, u_prev;
    Device* dev = nullptr;
};

// transcription (family.cpp)
bool build_structure(const nmpc_structure& s, Structure& out, std::string& err);
// SymCholesky (symbolic.cpp)
void symbolic_analyze(const Structure& st, Symbolic& sym);
// Update-block pool offsets for the given per-supernode execution steps.
void update_block_pool(const Symbolic& sym, const std::vector<int>& lev, std::vector<int64_t>& u_off,
                       int64_t& stored_u);
// device side (device.hip)
nmpc_status device_init(Problem& p, std::string& err);
void device_free(Problem& p);
nmpc_status device_set_parameters(Problem& p, std::string& err);
// Entry points on device pointers, ordered after the work on the caller's
// stream; the caller's stream is ordered after them (no host synchronization).
nmpc_status device_set_parameters_dev(Problem& p, const double* x0, const double* setpoint, const double* traj,
                                     const double* u_prev, void* caller, std::string& err);
nmpc_status device_get_solution_dev(const Problem& p, double* y, double* lam, double* omega_d, double* zl,
                                    double* zu, double* u1, double* x1, void* caller, std::string& err);
nmpc_status device_adjoint_dev(Problem& p, const double* seed_u1, const double* seed_obj, double* gx0, double* gsp,
                               double* gtraj, double* gup, void* caller, std::string& err);
nmpc_status device_solve(Problem& p, int warm, const nmpc_options& o, nmpc_result& r, std::string& err);
// Closed loop on the device: per step the parameter update from the held
// solution and `passes` passes in one captured graph, then passes until done.
nmpc_status device_closed_loop(Problem& p, int steps, const double* traj, const double* noise, double* u_out,
                               double* x_out, int passes, const nmpc_options& o, void* caller_stream,
                               int* steps_done, int* iters_total, std::string& err);
nmpc_status device_get_iterate(const Problem& p, double* y, double* s, double* om, double* be,
                               double* zl, double* zu, std::string& err);
nmpc_status device_get_first_stage(const Problem& p, double* u1, double* x1, std::string& err);
nmpc_status device_set_iterate(Problem& p, const double* y, const double* s, const double* om,
                               const double* be, const double* zl, const double* zu, std::string& err);
nmpc_status device_eval(Problem& p, const double* y, const double* lam, const double* lam_d, double* f,
                        double* grad, double* c, double* d, double* jv, double* wv, std::string& err);
nmpc_status device_factor(Problem& p, const double* kv, double eta, int32_t* ok, double* lv,
                          std::string& err);
nmpc_status device_linear_solve(Problem& p, const double* b, double* x, std::string& err);
nmpc_status device_assemble(Problem& p, double mu, double* kv, double* rhs, std::string& err);
nmpc_status device_adjoint(Problem& p, const double* seed_u1, double seed_obj, double* gx0, double* gsp,
                           double* gtraj, double* gup, std::string& err);
nmpc_status device_jacobian_u1_x0(Problem& p, double* jac, std::string& err);
// Allocation-free Jacobian: its vectors live in a fixed per-GPU device buffer
// of kNoAllocScratchBytes; noalloc_scratch_bytes is what a problem needs there
// (host arithmetic on the structure and the symbolic analysis).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
size_t noalloc_scratch_bytes(const Problem& p);
nmpc_status device_jacobian_u1_x0_noalloc(Problem& p, double* jac, void* caller, std::string& err);
void device_invalidate_adjoint(Problem& p);
nmpc_status device_autotune(Problem& p, int reps, int* changed, std::string& err);
nmpc_status batch_create(const std::vector<Problem*>& ps, Batch*& out, std::string& err);
void batch_free(Batch* b);
int batch_size(const Batch& b);
nmpc_status batch_solve(Batch& b, int warm, const nmpc_options& o, nmpc_result* res, std::string& err);
bool device_present();

}  // namespace nmpc

#endif
