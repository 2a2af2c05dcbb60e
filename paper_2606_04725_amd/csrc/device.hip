// Device buffers of a problem, batches of problems, and the host side of
// Algorithm 2.
//
// Every step of an iteration runs on the GPU: model evaluation, residuals and
// optimality errors (eqs. 11, 27-28), condensed assembly (eqs. 14, 17), the
// supernodal factorization with inertia correction (eqs. 12-13, 20-21), the
// forward/back solves (eqs. 22-25), recovery of the other directions, the
// fraction-to-boundary rule and the line search (eq. 26).  The scalar
// decisions (barrier update, regularization, step acceptance) are taken on the
// device too, per instance, by the decision kernels.  The host enqueues passes:
// in one pass every running instance moves through one Newton iteration (or
// one more factorization attempt, or one more trial point, when its last one
// failed), so instances of a batch never wait for each other.  A pass needs no
// host decision, so it is captured once as a HIP graph and replayed; after
// each pass the host reads one integer, the number of instances still running.
//
// A problem's own solve is a batch of one; a user batch groups the device state
// of several analyzed problems and runs the same passes over all of them, so
// an instance's arithmetic is the same alone or batched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace nmpc {

static_assert(kFilterCapMax == kFilterCapacity, "filter capacity of the options check and of the device storage");

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return e_ == hipErrorOutOfMemory ? NMPC_ERR_OOM : NMPC_ERR_HIP;           \
        }                                                                             \
    } while (0)

// Launch schedule of one instance: a list of steps.  A group step is a list of
// groups (supernodes walked in order by one workgroup, in sched_nodes order);
// a large-supernode step is a task list for one of the kernels of the
// multi-workgroup path (BigKind).
enum StepKind : int { kStepGroupFactor = 100, kStepGroupFwd = 101, kStepGroupBwd = 102 };
struct LocalGroup {
    int begin, end;
    size_t lds_factor, lds_solve;   // shared-memory bytes the group needs
};
struct Step {
    int kind = 0;
    int variant = 0;                // front-kernel variant of a group factor step (autotuned)
    std::vector<LocalGroup> groups;
    std::vector<int4> tasks;        // x (the instance) is filled in by the batch
    size_t lds = 0;                 // shared memory of a large-supernode solve kernel
};

struct Device {
    const Problem* owner = nullptr;
    hipStream_t stream = nullptr;
    InstPtrs hI{};                 // host copy of the instance descriptor
    std::vector<Step> fac, fwd, bwd;
    std::vector<Step> fwd_rest;   // forward steps of the supernodes whose Newton-step forward solve is not fused
    int fac_launches = 0;          // kernel launches of one factorization
    int64_t stored_l = 0, nnzj = 0, nnzw = 0;
    std::vector<void*> allocs;
    Batch* self = nullptr;         // batch of one over this problem
    // sensitivities: factor of K at the returned iterate, kept until it changes
    bool adj_ready = false;
    double adj_eta = 0.0;
    double gamma_last = 1e-9;
    // ordering against a caller's stream (the entry points taking device pointers)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the nu seeds of the u1 / x0 Jacobian solved together: a batch whose
    // instances share this problem's factor, iterate and structure and own only
    // the vectors a sensitivity solve writes (contiguous, seed k at offset k size)
    Batch* seeds = nullptr;
    std::vector<Device*> seed_devs;
    double* seed_vals = nullptr;   // nu x (nu + 1) seeds
    double* seed_lam = nullptr;    // nu x m multipliers; row k's first nx entries are d u1_k / d x0
    // this GPU's fixed buffer of the allocation-free Jacobian (resolved at set-up)
    unsigned char* scratch = nullptr;
    // stage-model family: the generated kernels, loaded on this device
    hipModule_t mod = nullptr;
    hipFunction_t f_eval = nullptr, f_guess = nullptr, f_adj = nullptr;
    hipFunction_t f_reduce = nullptr;   // pattern models: sums the per-stage scratch after an evaluation
    double* gm_jac = nullptr;      // nu x nx: d u1 / d x0 mapped through the state rows' coefficients
};

// Kernels of one generated stage model as a batch launches them.
struct GenFns {
    hipFunction_t eval, guess, reduce;
    bool operator==(const GenFns& o) const { return eval == o.eval && guess == o.guess && reduce == o.reduce; }
};

// Emitted kernel launch of a batch schedule: a group launch (groups[off ..
// off + count)) or a large-supernode step (tasks[off .. off + count)).
struct BLaunch {
    int kind, off, count;
    bool lds;
    size_t bytes;
    int variant;
    int step;       // index of the instances' step it comes from
};

struct Batch {
    std::vector<Device*> members;
    int ninst = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    InstPtrs* dI = nullptr;
    Ctl* ctl = nullptr;
    IpmSpaces spaces{};
    Group* groups = nullptr;
    int4* tasks = nullptr;
    std::vector<BLaunch> fac, fwd, bwd, fwd_rest;
    bool has_distill = false, has_plate = false, has_reflux = false;
    // generated kernels of the stage models among the members (one entry per
    // distinct code object; each launch covers the batch, its kernels skip
    // instances with another tag)
    std::vector<GenFns> gen;
    int* running = nullptr;        // device: instances running, instances waiting for corrections,
                                   // instances whose HyKKT conjugate gradients run
    int* hrunning = nullptr;       // pinned copy
    Ctl* hctl = nullptr;           // pinned
    hipEvent_t ev[8] = {};
    // captured graphs, index timed + 2 * part: part 0 the pass, part 1 the
    // second-order corrections (replayed only when an instance waits for them)
    hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
    DevOpts graph_opts[4] = {};                       // options the graphs were captured with
    bool graph_failed[2] = {false, false};
    // closed loop on the device: the parameter update, the control-block reset
    // and a fixed number of passes, captured together (and what they were
    // captured with)
    hipGraph_t loop_graph = nullptr;
    hipGraphExec_t loop_exec = nullptr;
    struct LoopKey {
        DevOpts o;
        const void *traj, *noise, *u_out, *x_out;
        int passes;
    } loop_key{};
    int* loop_ctr = nullptr;       // device: index of the next step
    Ctl* loop_ctl = nullptr;       // pinned: the control block every step starts from
    std::vector<void*> allocs;
};

namespace {


inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

template <class T>
hipError_t dalloc(std::vector<void*>& allocs, T*& p, size_t count) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        allocs.push_back(v);
        p = static_cast<T*>(v);
    }
    return e;
}

template <class T>
hipError_t upload(std::vector<void*>& allocs, T*& p, const std::vector<T>& h) {
    hipError_t e = dalloc(allocs, p, h.size());
    if (e != hipSuccess) return e;
    if (!h.empty()) e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

template <class T>
hipError_t upload_c(std::vector<void*>& allocs, const T*& p, const std::vector<T>& h) {
    T* q = nullptr;
    hipError_t e = upload(allocs, q, h);
    p = q;
    return e;
}

DevOpts dev_opts(const nmpc_options& o) {
    DevOpts d;
    std::memset(&d, 0, sizeof(d));   // padding too: the struct is compared bytewise
    d.tol = o.tol;
    d.mu_min = o.mu_min;
    d.kappa_eps = o.kappa_eps;
    d.kappa_mu = o.kappa_mu;
    d.theta_mu = o.theta_mu;
    d.tau_min = o.tau_min;
    d.armijo = o.armijo;
    d.kappa_sigma = o.kappa_sigma;
    d.eta_first = o.eta_first;
    d.eta_min = o.eta_min;
    d.eta_max = o.eta_max;
    d.kp_first = o.kp_first;
    d.kp = o.kp;
    d.km = o.km;
    d.g_theta = o.filter_gamma_theta;
    d.g_phi = o.filter_gamma_phi;
    d.s_theta = o.filter_s_theta;
    d.s_phi = o.filter_s_phi;
    d.delta = o.filter_delta;
    d.amin_frac = o.alpha_min_frac;
    d.theta_max_fact = o.theta_max_fact;
    d.theta_min_fact = o.theta_min_fact;
    d.soc_kappa = o.soc_kappa;
    d.ls_max = o.ls_max;
    d.max_iter = o.max_iter;
    d.filter_cap = o.filter_cap;
    d.soc_max = o.soc_max;
    d.merit_fallback = o.merit_fallback;
    d.fixed_mu = o.fixed_mu;
    d.cg_tol = o.hykkt_cg_tol;
    d.cg_max = o.hykkt_cg_max;
    // each second-order correction would need its own conjugate-gradient
    // solve: HyKKT runs without them
    if (o.kkt == NMPC_KKT_HYKKT) d.soc_max = 0;
    return d;
}

size_t lds_limit_bytes() {
    int dev = 0, lds_max = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    return (size_t)lds_max;
}

void batch_release(Batch* B) {
    if (!B) return;
    for (int k = 0; k < 4; ++k) {
        if (B->exec[k]) (void)hipGraphExecDestroy(B->exec[k]);
        if (B->graph[k]) (void)hipGraphDestroy(B->graph[k]);
    }
    if (B->loop_exec) (void)hipGraphExecDestroy(B->loop_exec);
    if (B->loop_graph) (void)hipGraphDestroy(B->loop_graph);
    for (void* a : B->allocs) (void)hipFree(a);
    if (B->hrunning) (void)hipHostFree(B->hrunning);
    if (B->hctl) (void)hipHostFree(B->hctl);
    if (B->loop_ctl) (void)hipHostFree(B->loop_ctl);
    for (auto e : B->ev)
        if (e) (void)hipEventDestroy(e);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

// Build the device tables of a batch over the given instances.
nmpc_status batch_build(const std::vector<Device*>& members, hipStream_t stream, Batch*& out, std::string& err) {
    Batch* B = new Batch();
    B->members = members;
    B->ninst = (int)members.size();
    auto bail = [&](nmpc_status rc) {
        batch_release(B);
        out = nullptr;
        return rc;
    };
#define BTRY(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
            return bail(e_ == hipErrorOutOfMemory ? NMPC_ERR_OOM : NMPC_ERR_HIP);      \
        }                                                                              \
    } while (0)
    if (stream) {
        B->stream = stream;
    } else {
        BTRY(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
        B->own_stream = true;
    }
    const int ni = B->ninst;
    BTRY(dalloc(B->allocs, B->ctl, ni));
    std::vector<InstPtrs> hI(ni);
    for (int i = 0; i < ni; ++i) {
        hI[i] = members[i]->hI;
        hI[i].ctl = B->ctl + i;
        if (hI[i].family == NMPC_FAMILY_DISTILLATION) B->has_distill = true;
        if (hI[i].family == NMPC_FAMILY_HEATED_PLATE) B->has_plate = true;
        if (hI[i].family == NMPC_FAMILY_REFLUX_COLUMN) B->has_reflux = true;
        if (hI[i].family == NMPC_FAMILY_STAGE_MODEL) {
            const GenFns f{members[i]->f_eval, members[i]->f_guess, members[i]->f_reduce};
            if (f.eval && f.guess && std::find(B->gen.begin(), B->gen.end(), f) == B->gen.end())
                B->gen.push_back(f);
        }
    }
    BTRY(upload(B->allocs, B->dI, hI));
    // index spaces
    for (int k = 0; k < kNumSpaces; ++k) {
        std::vector<int32_t> binst, bfirst(ni + 1, 0);
        for (int i = 0; i < ni; ++i) {
            bfirst[i] = (int32_t)binst.size();
            const int nb = std::max(1, nblocks(space_size(hI[i], k)));
            for (int b = 0; b < nb; ++b) binst.push_back(i);
        }
        bfirst[ni] = (int32_t)binst.size();
        Space& sp = B->spaces.sp[k];
        sp.blocks = (int)binst.size();
        BTRY(upload_c(B->allocs, sp.binst, binst));
        BTRY(upload_c(B->allocs, sp.bfirst, bfirst));
    }
    // schedules: step j of the batch holds step j of every instance (the
    // forward lists aligned at the leaves, the backward lists at the roots), one
    // launch per kind; factor groups split by whether their fronts fit in shared
    // memory
    const size_t lim = lds_limit_bytes();
    std::vector<Group> gl;
    std::vector<int4> tl;
    auto merge = [&](std::vector<BLaunch>& dst, std::vector<Step> Device::*list) {
        size_t len = 0;
        for (auto* D : members) len = std::max(len, (D->*list).size());
        for (size_t j = 0; j < len; ++j) {
            std::vector<Group> g_lds, g_glob, g_sol;
            size_t b_lds = 0, b_sol = 0;
            int gkind = 0, variant = 0, vfront = -1;
            std::vector<std::vector<int4>> by_kind(32);
            std::vector<size_t> kind_lds(32, 0);
            for (int i = 0; i < ni; ++i) {
                const auto& L = members[i]->*list;
                if (j >= L.size()) continue;
                const Step& st = L[j];
                if (st.kind >= kStepGroupFactor) {
                    gkind = st.kind;
                    if (st.kind == kStepGroupFactor) {   // the variant tuned for the largest front
                        int mx = 0;
                        for (const auto& g : st.groups) mx = std::max<int>(mx, (int)g.lds_factor);
                        if (mx > vfront) {
                            vfront = mx;
                            variant = st.variant;
                        }
                    }
                    int slot = 0;
                    for (const auto& g : st.groups) {
                        if (st.kind == kStepGroupFactor) {
                            if (g.lds_factor <= lim) {
                                g_lds.push_back(Group{i, g.begin, g.end, 0});
                                b_lds = std::max(b_lds, g.lds_factor);
                            } else {
                                g_glob.push_back(Group{i, g.begin, g.end, slot++});
                            }
                        } else {
                            g_sol.push_back(Group{i, g.begin, g.end, 0});
                            b_sol = std::max(b_sol, g.lds_solve);
                        }
                    }
                } else {
                    for (int4 t : st.tasks) {
                        t.x = i;
                        by_kind[st.kind].push_back(t);
                    }
                    kind_lds[st.kind] = std::max(kind_lds[st.kind], st.lds);
                }
            }
            auto emit_groups = [&](const std::vector<Group>& g, int kind, bool lds, size_t bytes) {
                if (g.empty()) return;
                dst.push_back(BLaunch{kind, (int)gl.size(), (int)g.size(), lds, bytes, variant, (int)j});
                gl.insert(gl.end(), g.begin(), g.end());
            };
            emit_groups(g_lds, kStepGroupFactor, true, b_lds);
            emit_groups(g_glob, kStepGroupFactor, false, 0);
            emit_groups(g_sol, gkind, true, b_sol);
            for (int k = 0; k < 32; ++k) {
                if (by_kind[k].empty()) continue;
                dst.push_back(BLaunch{k, (int)tl.size(), (int)by_kind[k].size(), false, kind_lds[k], 0, (int)j});
                tl.insert(tl.end(), by_kind[k].begin(), by_kind[k].end());
            }
        }
    };
    merge(B->fac, &Device::fac);
    merge(B->fwd, &Device::fwd);
    merge(B->fwd_rest, &Device::fwd_rest);
    merge(B->bwd, &Device::bwd);
    BTRY(upload(B->allocs, B->groups, gl));
    BTRY(upload(B->allocs, B->tasks, tl));
    BTRY(linalg_configure(lim));   // the device maximum, so every batch's launches fit
    BTRY(dalloc(B->allocs, B->running, 3));
    BTRY(hipHostMalloc((void**)&B->hrunning, 3 * sizeof(int), hipHostMallocDefault));
    BTRY(hipHostMalloc((void**)&B->hctl, sizeof(Ctl) * ni, hipHostMallocDefault));
    for (auto& e : B->ev) BTRY(hipEventCreate(&e));
#undef BTRY
    out = B;
    return NMPC_OK;
}

// ---- building blocks ------------------------------------------------------------
void eval(Batch& B, bool full, int src, int pred) {
    if (B.has_distill) launch_eval_distill(full, src, pred, B.dI, B.spaces.sp[kSpN], B.stream);
    if (B.has_plate) launch_eval_plate(full, src, pred, B.dI, B.spaces.sp[kSpN], B.stream);
    if (B.has_reflux) launch_eval_reflux(full, src, pred, B.dI, B.spaces.sp[kSpN], B.stream);
    // stage models: one lane per (stage, max(ns, rps)) -> the max(n, ml) space
    // (ml = 2 H rps); a failed launch is left in hipGetLastError
    for (const auto& g : B.gen) {
        Space sp = B.spaces.sp[kSpMax];
        const InstPtrs* dI = B.dI;
        int fl = full ? 1 : 0;
        void* args[] = {&dI, &sp, &src, &pred, &fl};
        if (sp.blocks > 0)
            (void)hipModuleLaunchKernel(g.eval, sp.blocks, 1, 1, kBlock, 1, 1, 0, B.stream, args, nullptr);
        // pattern models: sum the instances' contributions (same space, grid-stride inside)
        void* rargs[] = {&dI, &sp, &pred, &fl};
        if (sp.blocks > 0 && g.reduce)
            (void)hipModuleLaunchKernel(g.reduce, sp.blocks, 1, 1, kBlock, 1, 1, 0, B.stream, rargs, nullptr);
    }
}

void cold_guess(Batch& B) {
    launch_cold_guess(B.dI, B.spaces.sp[kSpN], B.stream);
    for (const auto& g : B.gen) {
        Space sp = B.spaces.sp[kSpN];
        const InstPtrs* dI = B.dI;
        void* args[] = {&dI, &sp};
        if (sp.blocks > 0)
            (void)hipModuleLaunchKernel(g.guess, sp.blocks, 1, 1, kBlock, 1, 1, 0, B.stream, args, nullptr);
    }
}

void run_launch(Batch& B, const BLaunch& L, int pred, double eta_force, int which) {
    switch (L.kind) {
        case kStepGroupFactor:
            launch_factor_groups(L.lds, L.variant, pred, eta_force, B.dI, B.groups + L.off, L.count, L.bytes,
                                 B.stream);
            break;
        case kStepGroupFwd:
            launch_fwd_groups(pred, which, B.dI, B.groups + L.off, L.count, L.bytes, B.stream);
            break;
        case kStepGroupBwd:
            launch_bwd_groups(pred, which, B.dI, B.groups + L.off, L.count, L.bytes, B.stream);
            break;
        default:
            launch_big(L.kind, pred, eta_force, which, B.dI, B.tasks + L.off, L.count, L.bytes, B.stream);
    }
}

void factor_launches(Batch& B, int pred, double eta_force) {
    for (const auto& L : B.fac) run_launch(B, L, pred, eta_force, 0);
}

// which == 0 in a pass: the factorization already ran the forward solve of the
// fused supernodes, only the rest remain
void solve_launches(Batch& B, int pred, int which, bool fused_done = false) {
    for (const auto& L : fused_done ? B.fwd_rest : B.fwd) run_launch(B, L, pred, 0.0, which);
    for (const auto& L : B.bwd) run_launch(B, L, pred, 0.0, which);
}

// One pass of Algorithm 2 over every running instance.  An instance whose first
// trial point asks for second-order corrections waits in phase C; the
// corrections run in their own part, enqueued before the next pass only when
// some instance waits (most passes need none).
void enqueue_pass(Batch& B, const DevOpts& o, bool timed) {
    hipStream_t st = B.stream;
    auto mark = [&](int k) {
        if (timed) (void)hipEventRecord(B.ev[k], st);
    };
    mark(0);
    eval(B, true, kSrcIter, kPhA);
    launch_phaseA(B.dI, B.spaces, B.ninst, kPhA, o, true, st);
    mark(1);
    launch_assemble(B.dI, B.spaces, kPhB, st);
    mark(2);
    factor_launches(B, kPredFactor, 0.0);
    launch_decideF(B.dI, B.ninst, o, st);
    mark(3);
    solve_launches(B, kPhS, 0, true);
    launch_phaseE(B.dI, B.spaces, B.ninst, o, st);
    mark(4);
    launch_trial(B.dI, B.spaces, st);
    eval(B, false, kSrcTrial, kPhT);
    launch_phaseT(B.dI, B.spaces, B.ninst, o, st);
    launch_update(B.dI, B.spaces, B.ninst, o, B.running, st);
    mark(5);
}

// One pass of the HyKKT variant: as enqueue_pass up to the solve of the
// right-hand side, then conjugate gradients on the Schur complement (one
// iteration per host round trip, until no instance's CG runs; the device ends
// each at cg_max), the final solve, and the rest of the pass.
hipError_t enqueue_pass_hykkt(Batch& B, const DevOpts& o, bool timed) {
    hipStream_t st = B.stream;
    auto mark = [&](int k) {
        if (timed) (void)hipEventRecord(B.ev[k], st);
    };
    mark(0);
    eval(B, true, kSrcIter, kPhA);
    launch_phaseA(B.dI, B.spaces, B.ninst, kPhA, o, true, st);
    mark(1);
    launch_assemble(B.dI, B.spaces, kPhB, st);
    mark(2);
    factor_launches(B, kPredFactor, 0.0);
    launch_decideF(B.dI, B.ninst, o, st);
    mark(3);
    solve_launches(B, kPhS, 0, true);
    launch_hk_cg_start(B.dI, B.spaces, B.ninst, o, B.running + 2, st);
    for (int k = 0; k <= o.cg_max + 1; ++k) {
        hipError_t e = hipMemcpyAsync(B.hrunning + 2, B.running + 2, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        if (B.hrunning[2] == 0) break;
        launch_hk_cg_pre(B.dI, B.spaces, st);
        solve_launches(B, kPhS, 5);
        launch_hk_cg_post(B.dI, B.spaces, B.ninst, o, B.running + 2, st);
    }
    launch_hk_finish(B.dI, B.spaces, st);
    solve_launches(B, kPhS, 0, false);
    launch_phaseE(B.dI, B.spaces, B.ninst, o, st);
    mark(4);
    launch_trial(B.dI, B.spaces, st);
    eval(B, false, kSrcTrial, kPhT);
    launch_phaseT(B.dI, B.spaces, B.ninst, o, st);
    launch_update(B.dI, B.spaces, B.ninst, o, B.running, st);
    mark(5);
    return hipGetLastError();
}

void enqueue_corrections(Batch& B, const DevOpts& o, bool timed) {
    hipStream_t st = B.stream;
    if (timed) (void)hipEventRecord(B.ev[6], st);
    launch_soc_prepare(B.dI, B.spaces, st);
    solve_launches(B, kPhC, 4);
    launch_soc_step(B.dI, B.spaces, B.ninst, st);
    eval(B, false, kSrcTrial, kPhC);
    launch_soc_decide(B.dI, B.spaces, B.ninst, o, st);
    launch_update(B.dI, B.spaces, B.ninst, o, B.running, st);
    if (timed) (void)hipEventRecord(B.ev[7], st);
}

// Capture one part (0: the pass, 1: the corrections) as a graph, once per
// batch, timing mode and options.
hipError_t ensure_graph(Batch& B, const DevOpts& o, bool timed, int part) {
    const int k = (timed ? 1 : 0) + 2 * part;
    if (B.exec[k] && std::memcmp(&B.graph_opts[k], &o, sizeof(DevOpts)) == 0) return hipSuccess;
    if (B.exec[k]) {   // options changed: the kernels' arguments are part of the graph
        (void)hipGraphExecDestroy(B.exec[k]);
        (void)hipGraphDestroy(B.graph[k]);
        B.exec[k] = nullptr;
        B.graph[k] = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(B.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    if (part == 0) enqueue_pass(B, o, timed);
    else enqueue_corrections(B, o, timed);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(B.stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return e;
    }
    B.graph[k] = g;
    B.exec[k] = x;
    B.graph_opts[k] = o;
    return hipSuccess;
}

}  // namespace

// ---- fixed device buffer of the allocation-free Jacobian ---------------------------
// One seed's sensitivity vectors and the instance descriptor that points at
// them.  Each GPU holds its own copy from the library's first use on it until
// the process ends.  Host code uses the address hipGetSymbolAddress returns for
// the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mutex;
std::vector<unsigned char*> g_scratch_ptr;   // per device ordinal, resolved once

// Device address of the current device's copy of the buffer.
hipError_t scratch_address(unsigned char*& out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    }
    out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

// ==================================================================================
bool device_present() {
    int cnt = 0;
    if (hipGetDeviceCount(&cnt) != hipSuccess) return false;
    return cnt > 0;
}

void device_free(Problem& p) {
    if (!p.dev) return;
    Device& D = *p.dev;
    if (D.stream) (void)hipStreamSynchronize(D.stream);
    batch_release(D.self);
    batch_release(D.seeds);
    for (Device* c : D.seed_devs) delete c;
    for (void* a : D.allocs) (void)hipFree(a);
    if (D.mod) (void)hipModuleUnload(D.mod);
    if (D.ev_in) (void)hipEventDestroy(D.ev_in);
    if (D.ev_out) (void)hipEventDestroy(D.ev_out);
    if (D.stream) (void)hipStreamDestroy(D.stream);
    delete p.dev;
    p.dev = nullptr;
}

nmpc_status device_init(Problem& p, std::string& err) {
    if (p.dev) return NMPC_OK;
    const Structure& st = p.st;
    const Symbolic& sy = p.sym;
    p.dev = new Device();
    Device& D = *p.dev;
    D.owner = &p;
    auto bail = [&](nmpc_status rc) {
        device_free(p);
        return rc;
    };
#define DTRY(call)                                                                     \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
            return bail(e_ == hipErrorOutOfMemory ? NMPC_ERR_OOM : NMPC_ERR_HIP);      \
        }                                                                              \
    } while (0)
    DTRY(hipStreamCreateWithFlags(&D.stream, hipStreamNonBlocking));
    DTRY(scratch_address(D.scratch));
    DTRY(hipEventCreateWithFlags(&D.ev_in, hipEventDisableTiming));
    DTRY(hipEventCreateWithFlags(&D.ev_out, hipEventDisableTiming));
    InstPtrs& I = D.hI;
    I.family = st.desc.family;
    I.n = st.n;
    I.mc = st.m_c;
    I.md = st.m_d;
    I.ml = 2 * st.m_c + st.m_d;
    I.m = st.m_c + st.m_d;
    I.nx = st.nx;
    I.nu = st.nu;
    I.H = st.H;
    I.nnzk = (int64_t)sy.k_fpos.size();
    D.nnzj = (int64_t)st.jcol.size();
    D.nnzw = (int64_t)st.wrow.size();
    D.stored_l = sy.stored_l;
    const nmpc_structure& s = st.desc;
    I.dd.N = s.n_trays;
    I.dd.nx = s.n_trays + 2;
    I.dd.ns = s.n_trays + 4;
    I.dd.H = s.horizon;
    I.dd.fd = s.n_trays / 2;
    I.dd.hc = (s.control_horizon >= 1 && s.control_horizon < s.horizon) ? s.control_horizon : s.horizon;
    I.dc.dt = s.dt;
    I.dc.alpha = s.alpha;
    I.dc.F = s.feed_flow;
    I.dc.rho = s.move_penalty;
    I.ns = st.n / st.H;
    I.rps = st.nx;
    if (st.desc.family == NMPC_FAMILY_REFLUX_COLUMN) {
        I.rd = RefluxDims{s.n_trays, s.feed_tray, 2 * s.n_trays + 4, 2 * s.n_trays + 3, s.horizon};
        I.rc = RefluxConst{s.dt, s.alpha, s.feed_flow, s.distillate, s.feed_comp, s.hold_cond, s.hold_tray,
                           s.hold_reb, s.u_weight};
        I.rps = I.rd.rps;
        I.nsp = 2;
        I.ntr = 0;
    } else if (st.desc.family == NMPC_FAMILY_STAGE_MODEL) {
        const auto& M = st.gm;
        I.ns = M.ns;
        I.rps = M.rps;
        I.nsp = M.nsp;
        I.ntr = M.traj ? st.H : 0;
        I.gm = StageConst{s.dt, (unsigned long long)M.tag, nullptr, nullptr};
        DTRY(hipModuleLoadData(&D.mod, M.code.data()));
        DTRY(hipModuleGetFunction(&D.f_eval, D.mod, "nmpc_stage_eval"));
        DTRY(hipModuleGetFunction(&D.f_guess, D.mod, "nmpc_stage_guess"));
        DTRY(hipModuleGetFunction(&D.f_adj, D.mod, "nmpc_stage_adj"));
        if (M.scratch > 0) {
            if (hipModuleGetFunction(&D.f_reduce, D.mod, "nmpc_stage_reduce") != hipSuccess) {
                (void)hipGetLastError();
                err = "stage model: a model with per-stage scratch needs nmpc_stage_reduce in its code object";
                return bail(NMPC_ERR_INVALID_ARG);
            }
            DTRY(dalloc(D.allocs, I.gm.scratch, (size_t)st.H * (size_t)M.scratch));
        }
        hipDeviceptr_t abi_ptr = nullptr;
        size_t abi_bytes = 0;
        DTRY(hipModuleGetGlobal(&abi_ptr, &abi_bytes, D.mod, "nmpc_stage_abi"));
        unsigned int abi = 0;
        if (abi_bytes == sizeof(abi)) DTRY(hipMemcpyDtoH(&abi, abi_ptr, sizeof(abi)));
        if (abi != kStageAbi) {
            err = "stage model: the code object was generated for another library build (descriptor layout)";
            return bail(NMPC_ERR_INVALID_ARG);
        }
        if (!M.pc_minus_identity) {
            double* pc = nullptr;
            DTRY(dalloc(D.allocs, pc, M.pc.size()));
            DTRY(hipMemcpy(pc, M.pc.data(), M.pc.size() * sizeof(double), hipMemcpyHostToDevice));
            I.gm.pc = pc;
            DTRY(dalloc(D.allocs, D.gm_jac, (size_t)st.nu * st.nx));
        }
    } else if (st.desc.family == NMPC_FAMILY_HEATED_PLATE) {
        I.pd.G = s.grid;
        I.pd.nx = s.grid * s.grid;
        I.pd.ns = I.pd.nx + 16;
        I.pd.H = s.horizon;
        I.pd.q = s.grid / 4;
        I.pc.dt = s.dt;
        I.pc.kap = 0.5 * s.cond_slope;
        I.pc.inv_h2 = (double)(s.grid + 1) * (double)(s.grid + 1);
        I.nsp = I.pd.nx;
        I.ntr = 0;
    } else {
        I.nsp = 2;
        I.ntr = st.H;
    }
    // Supernode classes.  Small: the front fits in shared memory (one workgroup
    // factors it there).  Medium: it does not, but has at most kMediumFront rows
    // (one workgroup factors it in a global buffer).  Large: the multi-workgroup
    // path works on it in place.  Solves use one workgroup when the panel fits
    // in shared memory, the multi-workgroup path otherwise.
    const size_t lim = lds_limit_bytes();
    const int nsn = sy.nsn;
    std::vector<char> big_fac(nsn, 0), big_sol(nsn, 0);
    auto rows_of = [&](int sn) { return (int64_t)(sy.sn_rows_ptr[sn + 1] - sy.sn_rows_ptr[sn]); };
    auto width_of = [&](int sn) { return (int64_t)(sy.sn_ptr[sn + 1] - sy.sn_ptr[sn]); };
    // a shared-memory front is its packed lower triangle; a global one is square
    auto packed_bytes = [&](int sn) {
        const size_t mr = (size_t)rows_of(sn);
        return mr * (mr + 1) / 2 * sizeof(double);
    };
    // plus m values of the fused forward solve (shared memory in both cases)
    auto fac_bytes = [&](int sn) {
        const size_t mr = (size_t)rows_of(sn), vb = mr * sizeof(double);
        return packed_bytes(sn) + vb <= lim ? packed_bytes(sn) + vb : mr * (mr | 1) * sizeof(double);
    };
    auto sol_bytes = [&](int sn) {
        const size_t mr = (size_t)rows_of(sn), w = (size_t)width_of(sn);
        return (mr * (w | 1) + mr + 2 * w) * sizeof(double);
    };
    int medium_max = 0;
    for (int sn = 0; sn < nsn; ++sn) {
        const int64_t mr = rows_of(sn);
        big_fac[sn] = fac_bytes(sn) > lim && mr > kMediumFront;
        big_sol[sn] = sol_bytes(sn) > lim;
        if (!big_fac[sn] && fac_bytes(sn) > lim) medium_max = std::max<int>(medium_max, (int)mr);
    }
    // Fused forward solves: a supernode whose children all run it runs the
    // Newton step's forward solve with its factorization (their update vectors
    // are ready by then): a one-workgroup front right after it, a large front
    // panel by panel.  A one-workgroup front whose solve needs the large path
    // keeps the separate solve.
    std::vector<int32_t> fused(nsn, 0);
    for (int Lv = 0; Lv < sy.depth; ++Lv)
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) {
            const int32_t sn = sy.level_list[i];
            bool ok = big_fac[sn] || !big_sol[sn];
            for (int c = sy.child_ptr[sn]; ok && c < sy.child_ptr[sn + 1]; ++c) ok = fused[sy.child_list[c]] != 0;
            fused[sn] = ok ? 1 : 0;
        }
    // Schedule: per level (bottom-up) one group step for its small and medium
    // supernodes and the step sequence of the large path for its large ones; the
    // top levels that hold at most kTailWidth supernodes (a chain), none large, form a
    // single group walked by one workgroup (a chain costs one launch).
    constexpr int kTailWidth = 1;
    auto level_all_small = [&](int Lv) {
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i)
            if (big_fac[sy.level_list[i]] || big_sol[sy.level_list[i]]) return false;
        return true;
    };
    int tail = sy.depth;
    while (tail > 0 && sy.level_ptr[tail] - sy.level_ptr[tail - 1] <= kTailWidth && level_all_small(tail - 1)) --tail;
    if (sy.depth - tail < 2) tail = sy.depth;
    std::vector<int32_t> nodes;
    auto make_group = [&](const std::vector<int32_t>& sns) {
        LocalGroup g{(int)nodes.size(), 0, 0, 0};
        for (int32_t sn : sns) {
            nodes.push_back(sn);
            g.lds_factor = std::max(g.lds_factor, fac_bytes(sn));
            g.lds_solve = std::max(g.lds_solve, sol_bytes(sn));
        }
        g.end = (int)nodes.size();
        return g;
    };
    auto ceil_div = [](int64_t a, int64_t b) { return (int)((a + b - 1) / b); };
    const int RB = big_row_block(), TL = big_tile(), SR = big_solve_rows(), SC = big_solve_cols(), CH = big_chunk();
    auto push = [&](std::vector<Step>& dst, int kind, std::vector<int4>&& t, size_t lds = 0) {
        if (t.empty()) return;
        Step stp;
        stp.kind = kind;
        stp.tasks = std::move(t);
        stp.lds = lds;
        dst.push_back(std::move(stp));
    };
    auto big_factor_steps = [&](const std::vector<int32_t>& bigs) {
        std::vector<int4> t;
        for (int32_t sn : bigs)
            for (int j = 0; j < rows_of(sn); ++j) t.push_back(int4{0, sn, j, 0});
        push(D.fac, kBigInit, std::move(t));
        int maxch = 0;
        for (int32_t sn : bigs) maxch = std::max(maxch, sy.child_ptr[sn + 1] - sy.child_ptr[sn]);
        for (int r = 0; r < maxch; ++r) {
            std::vector<int4> e;
            for (int32_t sn : bigs) {
                if (sy.child_ptr[sn] + r >= sy.child_ptr[sn + 1]) continue;
                const int c = sy.child_list[sy.child_ptr[sn] + r];
                const int nc = (int)(rows_of(c) - width_of(c));
                for (int jc = 0; jc < nc; ++jc) e.push_back(int4{0, sn, r, jc});
            }
            push(D.fac, kBigExtend, std::move(e));
        }
        int64_t wmax = 0;
        for (int32_t sn : bigs) wmax = std::max(wmax, width_of(sn));
        for (int64_t kb = 0; kb < wmax; kb += kBigOuter) {
            for (int64_t ki = kb; ki < std::min<int64_t>(wmax, kb + kBigOuter); ki += kBigPanel) {
                std::vector<int4> po, tr, up;
                for (int32_t sn : bigs) {
                    const int64_t w = width_of(sn), m = rows_of(sn);
                    if (ki >= w) continue;
                    const int64_t pw = std::min<int64_t>(kBigPanel, w - ki);
                    po.push_back(int4{0, sn, (int)ki, 0});
                    const int64_t below = m - ki - pw;
                    for (int rb = 0; rb < ceil_div(below, RB); ++rb) tr.push_back(int4{0, sn, (int)ki, rb});
                    const int64_t cend = std::min<int64_t>(w, kb + kBigOuter), t0 = ki + pw;
                    if (cend > t0) {   // the rest of the outer panel
                        const int trn = ceil_div(m - t0, TL), tcn = ceil_div(cend - t0, TL);
                        for (int ti = 0; ti < trn; ++ti)
                            for (int tj = 0; tj < tcn && tj <= ti; ++tj) up.push_back(int4{0, sn, (int)ki, ti * tcn + tj});
                    }
                }
                push(D.fac, kBigPotrf, std::move(po));
                push(D.fac, kBigTrsm, std::move(tr));
                push(D.fac, kBigUpdateInner, std::move(up));
            }
            std::vector<int4> up;
            for (int32_t sn : bigs) {
                const int64_t w = width_of(sn), m = rows_of(sn);
                if (kb >= w) continue;
                const int64_t kw = std::min<int64_t>(kBigOuter, w - kb);
                const int T = ceil_div(m - kb - kw, TL);
                for (int tt = 0; tt < T * (T + 1) / 2; ++tt) up.push_back(int4{0, sn, (int)kb, tt});
            }
            push(D.fac, kBigUpdate, std::move(up));
        }
    };
    std::vector<int32_t> tail_nodes;
    for (int Lv = tail; Lv < sy.depth; ++Lv)
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) tail_nodes.push_back(sy.level_list[i]);
    // The bottom levels where every supernode has at most one child and none is
    // large are chains: one workgroup walks each chain (leaf first in the
    // factorization and forward solve, root first in the backward solve), one
    // launch for all of those levels instead of one per level.
    auto chain_level = [&](int Lv) {
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) {
            const int32_t sn = sy.level_list[i];
            if (big_fac[sn] || big_sol[sn] || sy.child_ptr[sn + 1] - sy.child_ptr[sn] > 1) return false;
        }
        return true;
    };
    int chain_top = 0;
    while (chain_top < tail && chain_level(chain_top)) ++chain_top;
    if (chain_top < 2) chain_top = 0;
    // Update blocks: the pool is planned per execution step, and the chained
    // levels run as one step (a chain can reach its third level while another
    // is still at its first), so they count as one level there.
    std::vector<int64_t> u_off = sy.u_off;
    int64_t stored_u = sy.stored_u;
    if (chain_top > 0) {
        std::vector<int> lev(nsn, 0);
        for (int Lv = 0; Lv < sy.depth; ++Lv)
            for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i)
                lev[sy.level_list[i]] = std::max(Lv, chain_top - 1) - (chain_top - 1);
        update_block_pool(sy, lev, u_off, stored_u);
    }
    std::vector<std::vector<int32_t>> chains;   // leaf first
    if (chain_top > 0) {
        std::vector<char> has_parent(nsn, 0);
        for (int i = sy.level_ptr[0]; i < sy.level_ptr[chain_top]; ++i) {
            const int32_t sn = sy.level_list[i];
            for (int c = sy.child_ptr[sn]; c < sy.child_ptr[sn + 1]; ++c) has_parent[sy.child_list[c]] = 1;
        }
        for (int i = sy.level_ptr[0]; i < sy.level_ptr[chain_top]; ++i) {
            int32_t x = sy.level_list[i];
            if (has_parent[x]) continue;
            std::vector<int32_t> ch;
            while (true) {
                ch.push_back(x);
                if (sy.child_ptr[x + 1] == sy.child_ptr[x]) break;
                x = sy.child_list[sy.child_ptr[x]];
            }
            std::reverse(ch.begin(), ch.end());
            chains.push_back(std::move(ch));
        }
        Step gf, gs, gr;
        gf.kind = kStepGroupFactor;
        gs.kind = kStepGroupFwd;
        gr.kind = kStepGroupFwd;
        for (const auto& ch : chains) {
            gf.groups.push_back(make_group(ch));
            gs.groups.push_back(gf.groups.back());
            std::vector<int32_t> rest;
            for (int32_t sn : ch)
                if (!fused[sn]) rest.push_back(sn);
            if (!rest.empty()) gr.groups.push_back(make_group(rest));
        }
        D.fac.push_back(gf);
        D.fwd.push_back(gs);
        if (!gr.groups.empty()) D.fwd_rest.push_back(gr);
    }
    for (int Lv = chain_top; Lv < tail; ++Lv) {
        Step gf, gs, gr;
        gf.kind = kStepGroupFactor;
        gs.kind = kStepGroupFwd;
        gr.kind = kStepGroupFwd;
        std::vector<int32_t> bigs, bsol;
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) {
            const int32_t sn = sy.level_list[i];
            if (big_fac[sn]) bigs.push_back(sn);
            else gf.groups.push_back(make_group({sn}));
            if (big_sol[sn]) {
                bsol.push_back(sn);
            } else {
                gs.groups.push_back(make_group({sn}));
                if (!fused[sn]) gr.groups.push_back(gs.groups.back());
            }
        }
        if (!gf.groups.empty()) D.fac.push_back(gf);
        big_factor_steps(bigs);
        if (!gs.groups.empty()) D.fwd.push_back(gs);
        if (!gr.groups.empty()) D.fwd_rest.push_back(gr);
        int64_t nch = 0;
        for (int32_t sn : bsol) nch = std::max<int64_t>(nch, ceil_div(width_of(sn), CH));
        for (int c = 0; c < nch; ++c) {
            std::vector<int4> tri, gv;
            for (int32_t sn : bsol) {
                const int64_t w = width_of(sn), m = rows_of(sn), c0 = (int64_t)c * CH;
                if (c0 >= w) continue;
                tri.push_back(int4{0, sn, c, 0});
                const int64_t c1 = std::min<int64_t>(w, c0 + CH);
                for (int rb = 0; rb < ceil_div(m - c1, SR); ++rb) gv.push_back(int4{0, sn, c, rb});
            }
            std::vector<int4> tri_rest, gv_rest;   // the supernodes whose forward solve is not fused
            for (const int4& t : tri)
                if (!fused[t.y]) tri_rest.push_back(t);
            for (const int4& t : gv)
                if (!fused[t.y]) gv_rest.push_back(t);
            push(D.fwd_rest, kBigFwdTri, std::move(tri_rest));
            push(D.fwd_rest, kBigFwdGemv, std::move(gv_rest));
            push(D.fwd, kBigFwdTri, std::move(tri));
            push(D.fwd, kBigFwdGemv, std::move(gv));
        }
    }
    if (!tail_nodes.empty()) {
        Step gf, gs, gb;
        gf.kind = kStepGroupFactor;
        gs.kind = kStepGroupFwd;
        gb.kind = kStepGroupBwd;
        gf.groups.push_back(make_group(tail_nodes));
        gs.groups.push_back(gf.groups.back());
        std::vector<int32_t> rest;
        for (int32_t sn : tail_nodes)
            if (!fused[sn]) rest.push_back(sn);
        if (!rest.empty()) {
            Step gr;
            gr.kind = kStepGroupFwd;
            gr.groups.push_back(make_group(rest));
            D.fwd_rest.push_back(gr);
        }
        gb.groups.push_back(make_group(std::vector<int32_t>(tail_nodes.rbegin(), tail_nodes.rend())));
        D.fac.push_back(gf);
        D.fwd.push_back(gs);
        D.bwd.push_back(gb);
    }
    for (int Lv = tail - 1; Lv >= chain_top; --Lv) {
        Step gb;
        gb.kind = kStepGroupBwd;
        std::vector<int4> bb;
        std::vector<int32_t> bsol;
        for (int i = sy.level_ptr[Lv]; i < sy.level_ptr[Lv + 1]; ++i) {
            const int32_t sn = sy.level_list[i];
            if (big_sol[sn]) {
                bsol.push_back(sn);
                if (rows_of(sn) > width_of(sn))
                    for (int cb = 0; cb < ceil_div(width_of(sn), SC); ++cb) bb.push_back(int4{0, sn, cb, 0});
            } else {
                gb.groups.push_back(make_group({sn}));
            }
        }
        if (!gb.groups.empty()) D.bwd.push_back(gb);
        push(D.bwd, kBigBwdBelow, std::move(bb));
        int64_t nch = 0;
        for (int32_t sn : bsol) nch = std::max<int64_t>(nch, ceil_div(width_of(sn), CH));
        for (int64_t c = nch - 1; c >= 0; --c) {
            std::vector<int4> tri, gt;
            for (int32_t sn : bsol) {
                const int64_t w = width_of(sn), c0 = c * CH;
                if (c0 >= w) continue;
                tri.push_back(int4{0, sn, (int)c, 0});
                for (int cb = 0; cb < ceil_div(c0, SC); ++cb) gt.push_back(int4{0, sn, (int)c, cb});
            }
            push(D.bwd, kBigBwdTri, std::move(tri));
            push(D.bwd, kBigBwdGemvT, std::move(gt));
        }
    }
    if (!chains.empty()) {
        Step gb;
        gb.kind = kStepGroupBwd;
        for (const auto& ch : chains) gb.groups.push_back(make_group(std::vector<int32_t>(ch.rbegin(), ch.rend())));
        D.bwd.push_back(gb);
    }
    D.fac_launches = 0;
    for (const auto& stp : D.fac) {
        if (stp.kind != kStepGroupFactor) {
            ++D.fac_launches;
            continue;
        }
        bool in_lds = false, global = false;
        for (const auto& g : stp.groups) (g.lds_factor <= lim ? in_lds : global) = true;
        D.fac_launches += (int)in_lds + (int)global;
    }
    // front positions of the original entries: the large path keeps r + c (m | 1);
    // a one-workgroup front takes the layout of its group (packed lower in shared
    // memory; square with leading dimension m | 1 in a global buffer when any
    // front of the group is too large for shared memory), a diagonal entry
    // complemented (it takes + eta)
    std::vector<char> square(nsn, 0);
    for (const auto& stp : D.fac) {
        if (stp.kind != kStepGroupFactor) continue;
        for (const auto& g : stp.groups)
            if (g.lds_factor > lim)
                for (int i = g.begin; i < g.end; ++i) square[nodes[i]] = 1;
    }
    std::vector<int32_t> k_fpos = sy.k_fpos;
    for (int sn = 0; sn < nsn; ++sn) {
        if (big_fac[sn]) continue;
        const int64_t mr = rows_of(sn), ld = mr | 1;
        const bool packed = !square[sn];
        for (int32_t t = sy.k_ptr[sn]; t < sy.k_ptr[sn + 1]; ++t) {
            const int64_t pos = sy.k_fpos[t], r = pos % ld, c = pos / ld;
            const int64_t q = packed ? c * mr - c * (c + 1) / 2 + r : pos;
            k_fpos[t] = r == c ? ~(int32_t)q : (int32_t)q;
        }
    }
    // global front buffers for the medium groups of one step
    int max_global = 0;
    for (const auto& stp : D.fac) {
        if (stp.kind != kStepGroupFactor) continue;
        int cnt = 0;
        for (const auto& g : stp.groups)
            if (g.lds_factor > lim) ++cnt;
        max_global = std::max(max_global, cnt);
    }
    const int64_t gstride = max_global > 0 ? (int64_t)medium_max * (medium_max | 1) : 0;
    I.gstride = gstride;
    std::vector<void*>& A = D.allocs;
    DTRY(upload_c(A, I.jptr, st.jptr));
    DTRY(upload_c(A, I.jcol, st.jcol));
    DTRY(upload_c(A, I.jt_ptr, sy.jt_ptr));
    DTRY(upload_c(A, I.jt_slot, sy.jt_slot));
    DTRY(upload_c(A, I.jt_row, sy.jt_row));
    DTRY(upload_c(A, I.lb, st.lb));
    DTRY(upload_c(A, I.ub, st.ub));
    DTRY(upload_c(A, I.perm, sy.perm));
    DTRY(upload_c(A, I.S.sn_ptr, sy.sn_ptr));
    DTRY(upload_c(A, I.S.rows_ptr, sy.sn_rows_ptr));
    DTRY(upload_c(A, I.S.rows, sy.sn_rows));
    DTRY(upload_c(A, I.S.child_ptr, sy.child_ptr));
    DTRY(upload_c(A, I.S.child_list, sy.child_list));
    {
        std::vector<ChildRec> rec(sy.child_list.size());
        for (size_t k = 0; k < rec.size(); ++k) {
            const int c = sy.child_list[k];
            const int wc = sy.sn_ptr[c + 1] - sy.sn_ptr[c];
            rec[k] = ChildRec{u_off[c], sy.rel_off[c], sy.uv_off[c],
                              (int32_t)(sy.sn_rows_ptr[c + 1] - sy.sn_rows_ptr[c]) - wc, c};
        }
        DTRY(upload_c(A, I.S.child_rec, rec));
        std::vector<ChildRec> first((size_t)2 * std::max(sy.nsn, 1), ChildRec{0, 0, 0, 0, 0});
        for (int sn = 0; sn < sy.nsn; ++sn)
            for (int k = 0; k < 2 && sy.child_ptr[sn] + k < sy.child_ptr[sn + 1]; ++k)
                first[(size_t)2 * sn + k] = rec[(size_t)sy.child_ptr[sn] + k];
        DTRY(upload_c(A, I.S.first_recs, first));
    }
    DTRY(upload_c(A, I.S.l_off, sy.l_off));
    DTRY(upload_c(A, I.S.u_off, u_off));
    DTRY(upload_c(A, I.S.uv_off, sy.uv_off));
    DTRY(upload_c(A, I.S.rel_off, sy.rel_off));
    DTRY(upload_c(A, I.S.rel, sy.rel));
    DTRY(upload_c(A, I.S.k_ptr, sy.k_ptr));
    DTRY(upload_c(A, I.S.k_fpos, k_fpos));
    DTRY(upload_c(A, I.kcol_ptr, sy.kcol_ptr));
    DTRY(upload_c(A, I.S.sched_nodes, nodes));
    DTRY(upload_c(A, I.S.fused, fused));
    DTRY(upload_c(A, I.k_wslot, sy.k_wslot));
    DTRY(upload_c(A, I.k_diag, sy.k_diag));
    DTRY(upload_c(A, I.kc_ptr, sy.kc_ptr));
    DTRY(upload_c(A, I.kc_a, sy.kc_a));
    DTRY(upload_c(A, I.kc_b, sy.kc_b));
    DTRY(upload_c(A, I.kc_r, sy.kc_r));
    double *x0 = nullptr, *zF = nullptr, *up = nullptr, *setp = nullptr;
    DTRY(dalloc(A, x0, st.nx));
    DTRY(dalloc(A, zF, st.H));
    DTRY(dalloc(A, up, st.nu));
    DTRY(dalloc(A, setp, std::max<size_t>(2, p.setpoint.size())));
    I.x0 = x0;
    I.zF = zF;
    I.uprev = up;
    I.setp = setp;
    const int n = I.n, ml = I.ml, m = I.m, mc = I.mc, md = I.md;
    DTRY(dalloc(A, I.y, n)); DTRY(dalloc(A, I.s, ml)); DTRY(dalloc(A, I.om, ml)); DTRY(dalloc(A, I.be, ml));
    DTRY(dalloc(A, I.zl, n)); DTRY(dalloc(A, I.zu, n));
    DTRY(dalloc(A, I.c, mc)); DTRY(dalloc(A, I.d, md)); DTRY(dalloc(A, I.jv, D.nnzj)); DTRY(dalloc(A, I.wv, D.nnzw));
    DTRY(dalloc(A, I.grad, n)); DTRY(dalloc(A, I.fterm, n)); DTRY(dalloc(A, I.gtw, n)); DTRY(dalloc(A, I.sig, n));
    DTRY(dalloc(A, I.rhs, n)); DTRY(dalloc(A, I.dy, n)); DTRY(dalloc(A, I.xp, n));
    DTRY(dalloc(A, I.Q, ml)); DTRY(dalloc(A, I.r2, ml)); DTRY(dalloc(A, I.r4, ml)); DTRY(dalloc(A, I.qeff, m));
    DTRY(dalloc(A, I.vcomb, m));
    DTRY(dalloc(A, I.ds, ml)); DTRY(dalloc(A, I.dom, ml)); DTRY(dalloc(A, I.dbe, ml));
    DTRY(dalloc(A, I.dzl, n)); DTRY(dalloc(A, I.dzu, n)); DTRY(dalloc(A, I.yt, n)); DTRY(dalloc(A, I.st, ml));
    DTRY(dalloc(A, I.r1v, n)); DTRY(dalloc(A, I.r4s, ml)); DTRY(dalloc(A, I.vcomb_s, m)); DTRY(dalloc(A, I.rhs_s, n));
    DTRY(dalloc(A, I.dy_s, n)); DTRY(dalloc(A, I.ds_s, ml)); DTRY(dalloc(A, I.dom_s, ml)); DTRY(dalloc(A, I.dbe_s, ml));
    DTRY(dalloc(A, I.dzl_s, n)); DTRY(dalloc(A, I.dzu_s, n));
    DTRY(dalloc(A, I.kv, I.nnzk)); DTRY(dalloc(A, I.L, sy.stored_l)); DTRY(dalloc(A, I.U, stored_u));
    DTRY(dalloc(A, I.uvec, sy.stored_uv));
    DTRY(dalloc(A, I.adj_rhs, n)); DTRY(dalloc(A, I.adj_w, n));
    DTRY(dalloc(A, I.adj_out, st.nx + I.nsp + I.ntr + st.nu));
    DTRY(dalloc(A, I.adj_seed, st.nu + 1));
    DTRY(dalloc(A, I.adj_b, n)); DTRY(dalloc(A, I.adj_d, n)); DTRY(dalloc(A, I.adj_lam, m));
    DTRY(dalloc(A, I.adj_qr, m));
    DTRY(dalloc(A, I.bsum, n));
    DTRY(dalloc(A, I.hk_x, mc)); DTRY(dalloc(A, I.hk_r, mc)); DTRY(dalloc(A, I.hk_p, mc));
    DTRY(dalloc(A, I.hk_sp, mc)); DTRY(dalloc(A, I.hk_t, n)); DTRY(dalloc(A, I.hk_w, n));
    {
        // Hessian rows with both triangles, slots in increasing order per row
        std::vector<int32_t> cnt(n + 1, 0), wf_ptr(n + 1, 0);
        const size_t nw = st.wrow.size();
        for (size_t e = 0; e < nw; ++e) {
            cnt[st.wrow[e]]++;
            if (st.wrow[e] != st.wcol[e]) cnt[st.wcol[e]]++;
        }
        for (int j = 0; j < n; ++j) wf_ptr[j + 1] = wf_ptr[j] + cnt[j];
        std::vector<int32_t> wf_slot(wf_ptr[n]), wf_col(wf_ptr[n]), fill(wf_ptr.begin(), wf_ptr.end() - 1);
        for (size_t e = 0; e < nw; ++e) {
            const int r = st.wrow[e], c = st.wcol[e];
            wf_slot[fill[r]] = (int32_t)e;
            wf_col[fill[r]++] = c;
            if (r != c) {
                wf_slot[fill[c]] = (int32_t)e;
                wf_col[fill[c]++] = r;
            }
        }
        DTRY(upload_c(A, I.wf_ptr, wf_ptr));
        DTRY(upload_c(A, I.wf_slot, wf_slot));
        DTRY(upload_c(A, I.wf_col, wf_col));
    }
    int pblocks = 0;
    for (int k = 0; k < kNumSpaces; ++k) pblocks = std::max(pblocks, nblocks(space_size(I, k)));
    DTRY(dalloc(A, I.part, (size_t)kMaxQ * std::max(1, pblocks)));
    DTRY(dalloc(A, I.filter, (size_t)2 * kFilterCapMax));
    if (gstride > 0) DTRY(dalloc(A, I.gscratch, (size_t)gstride * max_global));
#undef DTRY
    std::vector<Device*> one{&D};
    nmpc_status rc = batch_build(one, D.stream, D.self, err);
    if (rc != NMPC_OK) return bail(rc);
    std::string e2;
    rc = device_set_parameters(p, e2);
    if (rc != NMPC_OK) {
        err = e2;
        return bail(rc);
    }
    return NMPC_OK;
}

nmpc_status device_set_parameters(Problem& p, std::string& err) {
    Device& D = *p.dev;
    const InstPtrs& I = D.hI;
    std::vector<double> sp(p.setpoint);
    if (sp.size() < 2) sp.resize(2, 0.0);
    HIP_TRY(hipMemcpyAsync((void*)I.x0, p.x0.data(), p.x0.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipMemcpyAsync((void*)I.zF, p.traj.data(), p.traj.size() * sizeof(double), hipMemcpyHostToDevice,
                           D.stream));
    HIP_TRY(hipMemcpyAsync((void*)I.uprev, p.u_prev.data(), p.u_prev.size() * sizeof(double),
                           hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipMemcpyAsync((void*)I.setp, sp.data(), sp.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    return NMPC_OK;
}

// ---- Algorithm 2 over a batch --------------------------------------------------------
nmpc_status batch_solve(Batch& B, int warm, const nmpc_options& o, nmpc_result* res, std::string& err) {
    const int ni = B.ninst;
    const DevOpts dop = dev_opts(o);
    const bool timed = o.timing != 0;
    const bool hyk = o.kkt == NMPC_KKT_HYKKT;
    hipStream_t st = B.stream;
    for (int i = 0; i < ni; ++i) {
        Ctl c{};
        c.hyk = hyk ? 1 : 0;
        c.hk_gamma = o.hykkt_gamma;
        c.mu = warm ? o.mu0_warm : o.mu0_cold;
        c.tau = std::max(o.tau_min, 1.0 - c.mu);
        c.E0 = INFINITY;
        c.filter_mu = std::nan("");
        c.nu = 1.0;
        c.gamma = o.gamma;
        c.status = kStatusRunning;
        c.phase = kPhA;
        B.hctl[i] = c;
        B.members[i]->adj_ready = false;
        B.members[i]->gamma_last = o.gamma;
    }
    HIP_TRY(hipMemcpyAsync(B.ctl, B.hctl, sizeof(Ctl) * ni, hipMemcpyHostToDevice, st));
    if (warm == 2) launch_shift(B.dI, B.spaces, st);   // shifted warm start
    if (warm && hyk) {   // a held Lifted-KKT iterate becomes a HyKKT one
        for (Device* m : B.members)
            if (!m->owner->iter_hyk && ni != 1) {
                err = "solve: HyKKT warm starts from Lifted-KKT iterates are for single problems";
                return NMPC_ERR_UNSUPPORTED;
            }
        if (!B.members[0]->owner->iter_hyk) launch_hk_from_lifted(B.dI, B.spaces, st);
    }
    if (!warm) {
        cold_guess(B);   // every stage: the measured state, the last control (stage models: their guess)
        launch_cold_start(B.dI, B.spaces, o.bound_push, o.slack_push, o.mu0_cold, false, st);
        eval(B, false, kSrcIter, kPredAll);
        launch_cold_start(B.dI, B.spaces, o.bound_push, o.slack_push, o.mu0_cold, true, st);
        HIP_TRY(hipGetLastError());
    }
    double ms[5] = {0, 0, 0, 0, 0};
    const int k = timed ? 1 : 0;
    bool use_graph = o.graph != 0 && !B.graph_failed[k] && !hyk;   // HyKKT: host-driven CG
    if (use_graph && (ensure_graph(B, dop, timed, 0) != hipSuccess ||
                      (o.soc_max > 0 && ensure_graph(B, dop, timed, 1) != hipSuccess))) {
        (void)hipGetLastError();
        B.graph_failed[k] = true;
        use_graph = false;
    }
    // every pass moves each running instance by one iteration, factorization
    // attempt or trial point; the method bounds all three
    const long max_passes = (long)(o.max_iter + 1) * (2L * o.ls_max + o.soc_max + 64) + 8;
    long passes = 0;
    int timing_lost = 0;
    bool corrections = false;   // an instance waits for second-order corrections
    while (true) {
        if (corrections) {
            if (use_graph) HIP_TRY(hipGraphLaunch(B.exec[k + 2], st));
            else enqueue_corrections(B, dop, timed);
        }
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(B.exec[k], st));
        } else if (hyk) {
            HIP_TRY(enqueue_pass_hykkt(B, dop, timed));
        } else {
            enqueue_pass(B, dop, timed);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipMemcpyAsync(B.hrunning, B.running, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        ++passes;
        if (timed) {
            bool lost = false;
            for (int ph = 0; ph < 6; ++ph) {
                if (ph == 5 && !corrections) break;
                float t = 0.0f;
                const hipError_t te = ph < 5 ? hipEventElapsedTime(&t, B.ev[ph], B.ev[ph + 1])
                                             : hipEventElapsedTime(&t, B.ev[6], B.ev[7]);
                if (te == hipSuccess) {
                    ms[ph < 5 ? ph : 4] += t;   // corrections count as line search
                } else {
                    (void)hipGetLastError();
                    lost = true;
                }
            }
            if (lost && use_graph) {   // events inside the graph did not time: launch eagerly from now on
                B.graph_failed[k] = true;
                use_graph = false;
                ++timing_lost;
            }
        }
        corrections = B.hrunning[1] > 0;
        if (B.hrunning[0] == 0) break;
        if (passes >= max_passes) {
            err = "solve: pass limit reached with instances still running";
            return NMPC_ERR_HIP;
        }
    }
    HIP_TRY(hipMemcpyAsync(B.hctl, B.ctl, sizeof(Ctl) * ni, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int worst = NMPC_OK;
    for (int i = 0; i < ni; ++i) {
        const Ctl& c = B.hctl[i];
        nmpc_result r{};
        r.status = c.status;
        r.iters = c.it;
        r.factorizations = c.factorizations;
        r.ls_trials = c.ls_trials;
        r.mu = c.mu;
        r.eta = c.eta;
        r.E0 = c.E0;
        r.objective = c.f;
        r.ms_eval = ms[0];
        r.ms_assemble = ms[1];
        r.ms_factor = ms[2];
        r.ms_solve = ms[3];
        r.ms_linesearch = ms[4];
        r.factor_launches = c.factorizations * B.members[i]->fac_launches;
        r.passes = (int)passes;
        r.timing_lost = timing_lost;
        r.cg_iters = c.cg_total;
        res[i] = r;
        worst = std::max(worst, (int)c.status);
    }
    return worst;
}

nmpc_status device_solve(Problem& p, int warm, const nmpc_options& o, nmpc_result& r, std::string& err) {
    return batch_solve(*p.dev->self, warm, o, &r, err);
}

// ---- closed loop on the device (Algorithm 1) ----------------------------------------------
namespace {

hipError_t join_in(Device& D, hipStream_t caller);
hipError_t join_out(Device& D, hipStream_t caller);

// Step k of the loop (k read from ctr): the held solution's first stage is the
// applied control and the predicted state (rows k of u_out / x_out); the next
// solve's parameters are x0 = x1 + noise row k clipped to the first stage's
// state bounds, u_prev = u1 and traj = traj row k (each optional).  One block.
__global__ void __launch_bounds__(kBlock)
k_loop_update(const InstPtrs* __restrict__ Ia, int* ctr, const double* __restrict__ traj,
              const double* __restrict__ noise, double* __restrict__ u_out, double* __restrict__ x_out) {
    const InstPtrs& I = Ia[0];
    __shared__ int k;
    if (threadIdx.x == 0) k = *ctr;
    __syncthreads();
    const int nx = I.nx, nu = I.nu;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const double x1 = I.y[i];
        if (x_out) x_out[(int64_t)k * nx + i] = x1;
        const double v = x1 + (noise ? noise[(int64_t)k * nx + i] : 0.0);
        const_cast<double*>(I.x0)[i] = fmin(fmax(v, I.lb[i]), I.ub[i]);
    }
    for (int j = threadIdx.x; j < nu; j += blockDim.x) {
        const double u1 = I.y[nx + j];
        if (u_out) u_out[(int64_t)k * nu + j] = u1;
        const_cast<double*>(I.uprev)[j] = u1;
    }
    if (traj)
        for (int t = threadIdx.x; t < I.H; t += blockDim.x) const_cast<double*>(I.zF)[t] = traj[(int64_t)k * I.H + t];
    __syncthreads();
    if (threadIdx.x == 0) *ctr = k + 1;
}

}  // namespace

nmpc_status device_closed_loop(Problem& p, int steps, const double* traj, const double* noise, double* u_out,
                               double* x_out, int passes, const nmpc_options& o, void* caller_stream,
                               int* steps_done, int* iters_total, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    const hipStream_t caller = static_cast<hipStream_t>(caller_stream);
    const hipStream_t st = B.stream;
    DevOpts dop = dev_opts(o);
    *steps_done = 0;
    *iters_total = 0;
    if (!B.loop_ctr) HIP_TRY(dalloc(B.allocs, B.loop_ctr, 1));
    if (!B.loop_ctl) HIP_TRY(hipHostMalloc((void**)&B.loop_ctl, sizeof(Ctl), hipHostMallocDefault));
    // the control block of a warm solve, the same for every step (pinned; the
    // captured copy reads it at each replay)
    {
        Ctl c{};
        c.mu = o.mu0_warm;
        c.tau = std::max(o.tau_min, 1.0 - c.mu);
        c.E0 = INFINITY;
        c.filter_mu = std::nan("");
        c.nu = 1.0;
        c.gamma = o.gamma;
        c.status = kStatusRunning;
        c.phase = kPhA;
        *B.loop_ctl = c;
    }
    Batch::LoopKey key;
    std::memset(&key, 0, sizeof(key));
    key.o = dop;
    key.traj = traj;
    key.noise = noise;
    key.u_out = u_out;
    key.x_out = x_out;
    key.passes = passes;
    if (!B.loop_exec || std::memcmp(&B.loop_key, &key, sizeof(key)) != 0) {
        if (B.loop_exec) (void)hipGraphExecDestroy(B.loop_exec);
        if (B.loop_graph) (void)hipGraphDestroy(B.loop_graph);
        B.loop_exec = nullptr;
        B.loop_graph = nullptr;
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_loop_update, dim3(1), dim3(kBlock), 0, st, B.dI, B.loop_ctr, traj, noise, u_out, x_out);
        (void)hipMemcpyAsync(B.ctl, B.loop_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st);
        for (int k = 0; k < passes; ++k) enqueue_pass(B, dop, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (e == hipSuccess) e = hipGraphInstantiate(&B.loop_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            B.loop_exec = nullptr;
            err = std::string("closed loop: graph capture failed: ") + hipGetErrorString(e);
            return NMPC_ERR_HIP;
        }
        B.loop_graph = g;
        B.loop_key = key;
    }
    const bool socs = o.soc_max > 0;
    if (ensure_graph(B, dop, false, 0) != hipSuccess || (socs && ensure_graph(B, dop, false, 1) != hipSuccess)) {
        err = "closed loop: pass graph capture failed";
        return NMPC_ERR_HIP;
    }
    D.adj_ready = false;
    D.gamma_last = o.gamma;
    HIP_TRY(join_in(D, caller));
    HIP_TRY(hipMemsetAsync(B.loop_ctr, 0, sizeof(int), st));   // not captured
    const long max_passes = (long)(o.max_iter + 1) * (2L * o.ls_max + o.soc_max + 64) + 8;
    int status = NMPC_OK;
    for (int k = 0; k < steps; ++k) {
        HIP_TRY(hipGraphLaunch(B.loop_exec, st));
        long npass = passes;
        while (true) {
            HIP_TRY(hipMemcpyAsync(B.hrunning, B.running, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (B.hrunning[0] == 0) break;
            if (npass >= max_passes) {
                err = "closed loop: pass limit reached";
                return NMPC_ERR_HIP;
            }
            if (B.hrunning[1] > 0) HIP_TRY(hipGraphLaunch(B.exec[2], st));
            HIP_TRY(hipGraphLaunch(B.exec[0], st));
            ++npass;
        }
        HIP_TRY(hipMemcpyAsync(B.hctl, B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *iters_total += B.hctl[0].it;
        status = B.hctl[0].status;
        *steps_done = k + 1;
        if (status != NMPC_OK) break;
    }
    // the host copies of the parameters follow the device's
    const InstPtrs& I = D.hI;
    HIP_TRY(hipMemcpyAsync(p.x0.data(), I.x0, p.x0.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(p.u_prev.data(), I.uprev, p.u_prev.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (traj) HIP_TRY(hipMemcpyAsync(p.traj.data(), I.zF, p.traj.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(join_out(D, caller));
    return status;
}

nmpc_status batch_create(const std::vector<Problem*>& ps, Batch*& out, std::string& err) {
    std::vector<Device*> members;
    for (Problem* p : ps) members.push_back(p->dev);
    return batch_build(members, nullptr, out, err);
}

void batch_free(Batch* b) {
    if (b && b->stream) (void)hipStreamSynchronize(b->stream);
    batch_release(b);
}

int batch_size(const Batch& b) { return b.ninst; }

// ---- single-problem entry points -------------------------------------------------------
namespace {

// Control block of a batch of one for the direct entry points (mu, gamma).
hipError_t set_ctl(Batch& B, double mu, double gamma) {
    Ctl c{};
    c.mu = mu;
    c.gamma = gamma;
    c.status = NMPC_OK;
    c.phase = kPhDone;
    B.hctl[0] = c;
    hipError_t e = hipMemcpyAsync(B.ctl, B.hctl, sizeof(Ctl), hipMemcpyHostToDevice, B.stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(B.stream);
}

// NumCholesky (eq. 20) of kv + eta I for a batch of one; returns the failure flag.
hipError_t factor_once(Batch& B, double eta, int& failed) {
    launch_set_fail(B.dI, 1, 0, B.stream);
    factor_launches(B, kPredAll, eta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(B.hctl, B.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, B.stream);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(B.stream);
    failed = B.hctl[0].fail;
    return e;
}

}  // namespace

nmpc_status device_get_iterate(const Problem& p, double* y, double* s, double* om, double* be, double* zl,
                               double* zu, std::string& err) {
    const InstPtrs& I = p.dev->hI;
    HIP_TRY(hipMemcpy(y, I.y, I.n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(s, I.s, I.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(om, I.om, I.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(be, I.be, I.ml * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(zl, I.zl, I.n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(zu, I.zu, I.n * sizeof(double), hipMemcpyDeviceToHost));
    return NMPC_OK;
}

nmpc_status device_get_first_stage(const Problem& p, double* u1, double* x1, std::string& err) {
    const InstPtrs& I = p.dev->hI;
    if (u1) HIP_TRY(hipMemcpy(u1, I.y + I.nx, I.nu * sizeof(double), hipMemcpyDeviceToHost));
    if (x1) HIP_TRY(hipMemcpy(x1, I.y, I.nx * sizeof(double), hipMemcpyDeviceToHost));
    return NMPC_OK;
}

nmpc_status device_set_iterate(Problem& p, const double* y, const double* s, const double* om, const double* be,
                               const double* zl, const double* zu, std::string& err) {
    Device& D = *p.dev;
    const InstPtrs& I = D.hI;
    D.adj_ready = false;
    HIP_TRY(hipMemcpy(I.y, y, I.n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.s, s, I.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.om, om, I.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.be, be, I.ml * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.zl, zl, I.n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I.zu, zu, I.n * sizeof(double), hipMemcpyHostToDevice));
    return NMPC_OK;
}

nmpc_status device_eval(Problem& p, const double* y, const double* lam, const double* lam_d, double* f,
                        double* grad, double* c, double* d, double* jv, double* wv, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    const InstPtrs& I = D.hI;
    // stage the multipliers as a lifted omega: omega+ = lam, omega- = 0, omega_d = lam_d
    std::vector<double> om(I.ml, 0.0);
    for (int r = 0; r < I.mc; ++r) om[r] = lam[r];
    for (int r = 0; r < I.md; ++r) om[2 * I.mc + r] = lam_d[r];
    HIP_TRY(hipMemcpyAsync(I.yt, y, I.n * sizeof(double), hipMemcpyHostToDevice, B.stream));
    HIP_TRY(hipMemcpyAsync(I.dom, om.data(), I.ml * sizeof(double), hipMemcpyHostToDevice, B.stream));
    eval(B, true, kSrcUser, kPredAll);
    HIP_TRY(hipGetLastError());
    std::vector<double> ft(I.n);
    HIP_TRY(hipMemcpyAsync(ft.data(), I.fterm, I.n * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (grad) HIP_TRY(hipMemcpyAsync(grad, I.grad, I.n * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (c) HIP_TRY(hipMemcpyAsync(c, I.c, I.mc * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (d && I.md) HIP_TRY(hipMemcpyAsync(d, I.d, I.md * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (jv) HIP_TRY(hipMemcpyAsync(jv, I.jv, D.nnzj * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (wv) HIP_TRY(hipMemcpyAsync(wv, I.wv, D.nnzw * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    HIP_TRY(hipStreamSynchronize(B.stream));
    if (f) {
        double acc = 0.0;
        for (double v : ft) acc += v;
        *f = acc;
    }
    return NMPC_OK;
}

nmpc_status device_factor(Problem& p, const double* kv, double eta, int32_t* ok, double* lv, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    D.adj_ready = false;
    HIP_TRY(hipMemcpyAsync(D.hI.kv, kv, D.hI.nnzk * sizeof(double), hipMemcpyHostToDevice, B.stream));
    int failed = 0;
    HIP_TRY(factor_once(B, eta, failed));
    *ok = failed ? 0 : 1;
    if (lv) HIP_TRY(hipMemcpy(lv, D.hI.L, D.stored_l * sizeof(double), hipMemcpyDeviceToHost));
    return NMPC_OK;
}

nmpc_status device_linear_solve(Problem& p, const double* b, double* x, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    HIP_TRY(hipMemcpyAsync(D.hI.yt, b, D.hI.n * sizeof(double), hipMemcpyHostToDevice, B.stream));
    solve_launches(B, kPredAll, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(x, D.hI.dzl, D.hI.n * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    HIP_TRY(hipStreamSynchronize(B.stream));
    return NMPC_OK;
}

namespace {
// eval, G^T omega and the condensed system at the handle's iterate
hipError_t assemble_here(Device& D, double mu) {
    Batch& B = *D.self;
    hipError_t e = set_ctl(B, mu, D.gamma_last);
    if (e != hipSuccess) return e;
    eval(B, true, kSrcIter, kPredAll);
    DevOpts unused{};
    launch_phaseA(B.dI, B.spaces, 1, kPredAll, unused, false, B.stream);
    launch_assemble(B.dI, B.spaces, kPredAll, B.stream);
    return hipGetLastError();
}
}  // namespace

nmpc_status device_assemble(Problem& p, double mu, double* kv, double* rhs, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    D.adj_ready = false;
    HIP_TRY(assemble_here(D, mu));
    if (kv) HIP_TRY(hipMemcpyAsync(kv, D.hI.kv, D.hI.nnzk * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    if (rhs) HIP_TRY(hipMemcpyAsync(rhs, D.hI.rhs, D.hI.n * sizeof(double), hipMemcpyDeviceToHost, B.stream));
    HIP_TRY(hipStreamSynchronize(B.stream));
    return NMPC_OK;
}

void device_invalidate_adjoint(Problem& p) {
    if (p.dev) p.dev->adj_ready = false;
}

namespace {

constexpr int kAdjRefine = 2;   // refinement steps per sensitivity solve

// Assemble and factor K at the handle's iterate (inertia correction as in the solve).
nmpc_status adjoint_prepare(Problem& p, std::string& err) {
    Device& D = *p.dev;
    if (D.adj_ready) return NMPC_OK;
    Batch& B = *D.self;
    HIP_TRY(assemble_here(D, 1.0));   // mu only enters r2, which the sensitivities do not use
    int failed = 0;
    double eta = 0.0;
    HIP_TRY(factor_once(B, 0.0, failed));
    if (failed) {
        nmpc_options o;
        nmpc_default_options(&o);
        eta = o.eta_first;
        while (true) {
            HIP_TRY(factor_once(B, eta, failed));
            if (!failed) break;
            eta *= o.kp_first;
            if (eta > o.eta_max) {
                err = "adjoint: the condensed matrix at the solution could not be factored";
                return NMPC_ERR_INVALID_ARG;
            }
        }
    }
    D.adj_eta = eta;
    D.adj_ready = true;
    return NMPC_OK;
}

// Sensitivity solve for the seed already placed in adj_seed (on the library's
// stream): rhs, solve, refinement, parameter contractions into adj_out.
nmpc_status adjoint_run(Problem& p, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    if (p.st.nu > kMaxSeed) {
        err = "adjoint: too many controls per stage";
        return NMPC_ERR_UNSUPPORTED;
    }
    launch_adj_seed(B.dI, B.spaces.sp[kSpN], B.stream);
    solve_launches(B, kPredAll, 2);
    // refinement against the uncondensed system: the condensed matrix rounds the
    // curvature next to the lifted weights, the uncondensed residual does not
    launch_adj_refine(0, B.dI, B.spaces, D.adj_eta, B.stream);
    for (int r = 0; r < kAdjRefine; ++r) {
        launch_adj_refine(1, B.dI, B.spaces, D.adj_eta, B.stream);
        solve_launches(B, kPredAll, 3);
        launch_adj_refine(2, B.dI, B.spaces, D.adj_eta, B.stream);
    }
    if (D.hI.family == NMPC_FAMILY_STAGE_MODEL) {
        const InstPtrs* dI = B.dI;
        void* args[] = {&dI};
        const int nout = D.hI.nx + D.hI.nsp + D.hI.ntr + D.hI.nu;
        HIP_TRY(hipModuleLaunchKernel(D.f_adj, (nout + kBlock - 1) / kBlock, 1, 1, kBlock, 1, 1, 0, B.stream, args,
                                      nullptr));
    } else {
        launch_adj_gather(B.dI, D.hI.family, D.hI.nx, B.stream);
    }
    HIP_TRY(hipGetLastError());
    return NMPC_OK;
}

nmpc_status adjoint_apply(Problem& p, const double* seed_u1, double seed_obj, std::vector<double>& out,
                          std::string& err) {
    Device& D = *p.dev;
    const Structure& st = p.st;
    std::vector<double> sb(st.nu + 1, 0.0);
    for (int j = 0; j < st.nu; ++j) sb[j] = seed_u1 ? seed_u1[j] : 0.0;
    sb[st.nu] = seed_obj;
    HIP_TRY(hipMemcpyAsync(D.hI.adj_seed, sb.data(), sb.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    nmpc_status rc = adjoint_run(p, err);
    if (rc != NMPC_OK) return rc;
    out.resize(st.nx + D.hI.nsp + D.hI.ntr + st.nu);
    HIP_TRY(hipMemcpyAsync(out.data(), D.hI.adj_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    HIP_TRY(hipStreamSynchronize(D.stream));
    return NMPC_OK;
}

// The library's stream waits for the work already on the caller's stream ...
hipError_t join_in(Device& D, hipStream_t caller) {
    hipError_t e = hipEventRecord(D.ev_in, caller);
    return e != hipSuccess ? e : hipStreamWaitEvent(D.stream, D.ev_in, 0);
}

// ... and the caller's stream waits for the library's work enqueued since.
hipError_t join_out(Device& D, hipStream_t caller) {
    hipError_t e = hipEventRecord(D.ev_out, D.stream);
    return e != hipSuccess ? e : hipStreamWaitEvent(caller, D.ev_out, 0);
}

hipError_t copy_d2d(double* dst, const double* src, size_t n, hipStream_t st) {
    return (dst && src && n) ? hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st) : hipSuccess;
}

}  // namespace

nmpc_status device_adjoint(Problem& p, const double* seed_u1, double seed_obj, double* gx0, double* gsp,
                           double* gtraj, double* gup, std::string& err) {
    nmpc_status rc = adjoint_prepare(p, err);
    if (rc != NMPC_OK) return rc;
    std::vector<double> out;
    rc = adjoint_apply(p, seed_u1, seed_obj, out, err);
    if (rc != NMPC_OK) return rc;
    const Structure& st = p.st;
    const int nsp = p.dev->hI.nsp, ntr = p.dev->hI.ntr;
    auto o = out.begin();
    if (gx0) std::copy(o, o + st.nx, gx0);
    if (gsp) std::copy(o + st.nx, o + st.nx + nsp, gsp);
    if (gtraj && ntr) std::copy(o + st.nx + nsp, o + st.nx + nsp + ntr, gtraj);
    if (gup) std::copy(o + st.nx + nsp + ntr, o + st.nx + nsp + ntr + st.nu, gup);
    return p.dev->adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

nmpc_status device_set_parameters_dev(Problem& p, const double* x0, const double* setpoint, const double* traj,
                                     const double* u_prev, void* caller_stream, std::string& err) {
    const hipStream_t caller = static_cast<hipStream_t>(caller_stream);
    Device& D = *p.dev;
    const InstPtrs& I = D.hI;
    HIP_TRY(join_in(D, caller));
    // the parameter buffers are read-only for the kernels, owned by the library
    HIP_TRY(copy_d2d(const_cast<double*>(I.x0), x0, (size_t)I.nx, D.stream));
    HIP_TRY(copy_d2d(const_cast<double*>(I.setp), setpoint, (size_t)I.nsp, D.stream));
    HIP_TRY(copy_d2d(const_cast<double*>(I.zF), traj, (size_t)I.ntr, D.stream));
    HIP_TRY(copy_d2d(const_cast<double*>(I.uprev), u_prev, (size_t)I.nu, D.stream));
    HIP_TRY(join_out(D, caller));
    return NMPC_OK;
}

nmpc_status device_get_solution_dev(const Problem& p, double* y, double* lam, double* omega_d, double* zl,
                                    double* zu, double* u1, double* x1, void* caller_stream, std::string& err) {
    const hipStream_t caller = static_cast<hipStream_t>(caller_stream);
    Device& D = *p.dev;
    const InstPtrs& I = D.hI;
    HIP_TRY(join_in(D, caller));
    HIP_TRY(copy_d2d(y, I.y, (size_t)I.n, D.stream));
    HIP_TRY(copy_d2d(zl, I.zl, (size_t)I.n, D.stream));
    HIP_TRY(copy_d2d(zu, I.zu, (size_t)I.n, D.stream));
    HIP_TRY(copy_d2d(u1, I.y + I.nx, (size_t)I.nu, D.stream));
    HIP_TRY(copy_d2d(x1, I.y, (size_t)I.nx, D.stream));
    if (lam || omega_d) launch_export_duals(D.self->dI, lam, omega_d, std::max(I.mc, I.md), D.stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(join_out(D, caller));
    return NMPC_OK;
}

nmpc_status device_adjoint_dev(Problem& p, const double* seed_u1, const double* seed_obj, double* gx0, double* gsp,
                               double* gtraj, double* gup, void* caller_stream, std::string& err) {
    const hipStream_t caller = static_cast<hipStream_t>(caller_stream);
    nmpc_status rc = adjoint_prepare(p, err);   // once per solution; may wait for the library's stream
    if (rc != NMPC_OK) return rc;
    Device& D = *p.dev;
    const InstPtrs& I = D.hI;
    HIP_TRY(join_in(D, caller));
    if (seed_u1) HIP_TRY(copy_d2d(I.adj_seed, seed_u1, (size_t)I.nu, D.stream));
    else HIP_TRY(hipMemsetAsync(I.adj_seed, 0, I.nu * sizeof(double), D.stream));
    if (seed_obj) HIP_TRY(copy_d2d(I.adj_seed + I.nu, seed_obj, 1, D.stream));
    else HIP_TRY(hipMemsetAsync(I.adj_seed + I.nu, 0, sizeof(double), D.stream));
    rc = adjoint_run(p, err);
    if (rc != NMPC_OK) return rc;
    const size_t nx = I.nx, nsp = I.nsp, ntr = I.ntr;
    HIP_TRY(copy_d2d(gx0, I.adj_out, nx, D.stream));
    HIP_TRY(copy_d2d(gsp, I.adj_out + nx, nsp, D.stream));
    HIP_TRY(copy_d2d(gtraj, I.adj_out + nx + nsp, ntr, D.stream));
    HIP_TRY(copy_d2d(gup, I.adj_out + nx + nsp + ntr, (size_t)I.nu, D.stream));
    HIP_TRY(join_out(D, caller));
    return D.adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

namespace {

// The seed batch of the Jacobian (built once per problem): nu instance
// descriptors copied from the problem's, each with its own right-hand sides,
// solution, solve workspace (xp, update vectors, column sums) and multipliers.
nmpc_status seeds_build(Problem& p, std::string& err) {
    Device& D = *p.dev;
    if (D.seeds) return NMPC_OK;
    for (Device* c : D.seed_devs) delete c;   // an earlier attempt that failed
    D.seed_devs.clear();
    const int K = p.st.nu;
    const int64_t n = D.hI.n, m = D.hI.m, nuv = p.sym.stored_uv;
    const int64_t nout = p.st.nx + D.hI.nsp + D.hI.ntr + p.st.nu;
    double *xp, *bsum, *uvec, *rhs, *w, *b, *d, *qr, *out;
    HIP_TRY(dalloc(D.allocs, xp, K * n));
    HIP_TRY(dalloc(D.allocs, bsum, K * n));
    HIP_TRY(dalloc(D.allocs, uvec, K * std::max<int64_t>(nuv, 1)));
    HIP_TRY(dalloc(D.allocs, rhs, K * n));
    HIP_TRY(dalloc(D.allocs, w, K * n));
    HIP_TRY(dalloc(D.allocs, b, K * n));
    HIP_TRY(dalloc(D.allocs, d, K * n));
    HIP_TRY(dalloc(D.allocs, D.seed_lam, K * m));
    HIP_TRY(dalloc(D.allocs, qr, K * m));
    HIP_TRY(dalloc(D.allocs, out, K * nout));
    HIP_TRY(dalloc(D.allocs, D.seed_vals, (int64_t)K * (K + 1)));
    for (int k = 0; k < K; ++k) {
        Device* c = new Device();
        c->owner = &p;
        c->hI = D.hI;
        InstPtrs& I = c->hI;
        I.xp = xp + k * n;
        I.bsum = bsum + k * n;
        I.uvec = uvec + k * std::max<int64_t>(nuv, 1);
        I.adj_rhs = rhs + k * n;
        I.adj_w = w + k * n;
        I.adj_b = b + k * n;
        I.adj_d = d + k * n;
        I.adj_lam = D.seed_lam + k * m;
        I.adj_qr = qr + k * m;
        I.adj_out = out + k * nout;
        I.adj_seed = D.seed_vals + (int64_t)k * (K + 1);
        c->fac = D.fac;
        c->fwd = D.fwd;
        c->bwd = D.bwd;
        c->fwd_rest = D.fwd_rest;
        D.seed_devs.push_back(c);
    }
    const nmpc_status rc = batch_build(D.seed_devs, D.stream, D.seeds, err);
    if (rc != NMPC_OK) {   // the descriptors go; their vectors stay with the problem's allocations
        for (Device* c : D.seed_devs) delete c;
        D.seed_devs.clear();
    }
    return rc;
}

}  // namespace

// Row k of d u1 / d x0 is the sensitivity for the seed e_k (the same arithmetic
// as nmpc_adjoint with that seed): all nu seeds go through one sequence of
// launches, each launch covering every seed.
nmpc_status device_jacobian_u1_x0(Problem& p, double* jac, std::string& err) {
    nmpc_status rc = adjoint_prepare(p, err);
    if (rc != NMPC_OK) return rc;
    const Structure& st = p.st;
    if (st.nu > kMaxSeed) {
        err = "adjoint: too many controls per stage";
        return NMPC_ERR_UNSUPPORTED;
    }
    rc = seeds_build(p, err);
    if (rc != NMPC_OK) return rc;
    Device& D = *p.dev;
    Batch& S = *D.seeds;
    const int K = st.nu;
    std::vector<double> sv((size_t)K * (K + 1), 0.0);
    for (int k = 0; k < K; ++k) sv[(size_t)k * (K + 1) + k] = 1.0;
    HIP_TRY(hipMemcpyAsync(D.seed_vals, sv.data(), sv.size() * sizeof(double), hipMemcpyHostToDevice, D.stream));
    launch_adj_seed(S.dI, S.spaces.sp[kSpN], S.stream);
    solve_launches(S, kPredAll, 2);
    launch_adj_refine(0, S.dI, S.spaces, D.adj_eta, S.stream);
    for (int r = 0; r < kAdjRefine; ++r) {
        launch_adj_refine(1, S.dI, S.spaces, D.adj_eta, S.stream);
        solve_launches(S, kPredAll, 3);
        launch_adj_refine(2, S.dI, S.spaces, D.adj_eta, S.stream);
    }
    HIP_TRY(hipGetLastError());
    if (D.hI.gm.pc) {   // stage model whose state rows hold the previous states through a matrix
        launch_x0_map(D.seed_lam, D.hI.m, D.hI.gm.pc, D.gm_jac, st.nx, K, D.stream);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(jac, D.gm_jac, (size_t)K * st.nx * sizeof(double), hipMemcpyDeviceToHost, D.stream));
    } else {
        HIP_TRY(hipMemcpy2DAsync(jac, st.nx * sizeof(double), D.seed_lam, (size_t)D.hI.m * sizeof(double),
                                 st.nx * sizeof(double), K, hipMemcpyDeviceToHost, D.stream));
    }
    HIP_TRY(hipStreamSynchronize(D.stream));
    return D.adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

// ---- the Jacobian without allocation ------------------------------------------------
namespace {

// Offsets (bytes, 256-aligned) of one seed's vectors in the fixed buffer: the
// instance descriptor, then the vectors a sensitivity solve writes.
struct NoAllocLayout {
    size_t desc, xp, bsum, uvec, rhs, w, b, d, lam, qr, out, seed, total;
};

NoAllocLayout noalloc_layout(const Problem& p) {
    const Structure& st = p.st;
    const size_t n = (size_t)st.n, m = (size_t)(st.m_c + st.m_d);
    const size_t nsp = st.desc.family == NMPC_FAMILY_HEATED_PLATE ? (size_t)st.nx
                       : st.desc.family == NMPC_FAMILY_STAGE_MODEL ? (size_t)st.gm.nsp
                                                                   : 2;
    const size_t ntr = st.desc.family == NMPC_FAMILY_DISTILLATION || (st.desc.family == NMPC_FAMILY_STAGE_MODEL &&
                                                                      st.gm.traj)
                           ? (size_t)st.H
                           : 0;
    const size_t nout = (size_t)st.nx + nsp + ntr + (size_t)st.nu;
    const size_t nuv = std::max<size_t>((size_t)p.sym.stored_uv, 1);
    NoAllocLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.desc = take(sizeof(InstPtrs));
    L.xp = take(n * sizeof(double));
    L.bsum = take(n * sizeof(double));
    L.uvec = take(nuv * sizeof(double));
    L.rhs = take(n * sizeof(double));
    L.w = take(n * sizeof(double));
    L.b = take(n * sizeof(double));
    L.d = take(n * sizeof(double));
    L.lam = take(m * sizeof(double));
    L.qr = take(m * sizeof(double));
    L.out = take(nout * sizeof(double));
    L.seed = take(((size_t)st.nu + 1) * sizeof(double));
    L.total = off;
    return L;
}

// Places the scratch instance's descriptor and the seed e_k (objective seed 0).
__global__ void k_noalloc_seed(InstPtrs J, InstPtrs* dst, int k) {
    if (threadIdx.x == 0) *dst = J;
    for (int i = threadIdx.x; i <= J.nu; i += blockDim.x) J.adj_seed[i] = i == k ? 1.0 : 0.0;
}

}  // namespace

size_t noalloc_scratch_bytes(const Problem& p) { return noalloc_layout(p).total; }

// Row k of d u1 / d x0 as in device_jacobian_u1_x0 (seed e_k, the same kernels
// and refinement), one seed after another through the problem's own launch
// schedule, with the vectors the solves write in this GPU's fixed buffer.
nmpc_status device_jacobian_u1_x0_noalloc(Problem& p, double* jac, void* caller_stream, std::string& err) {
    const Structure& st = p.st;
    if (st.nu > kMaxSeed) {
        err = "adjoint: too many controls per stage";
        return NMPC_ERR_UNSUPPORTED;
    }
    const NoAllocLayout Lo = noalloc_layout(p);
    if (Lo.total > kNoAllocScratchBytes) {
        err = "jacobian_u1_x0_noalloc: the problem needs " + std::to_string(Lo.total) +
              " bytes of scratch, more than the fixed " + std::to_string(kNoAllocScratchBytes);
        return NMPC_ERR_UNSUPPORTED;
    }
    nmpc_status rc = adjoint_prepare(p, err);   // once per solution; may wait for the library's stream
    if (rc != NMPC_OK) return rc;
    Device& D = *p.dev;
    Batch& B = *D.self;
    if (!D.scratch) {
        err = "jacobian_u1_x0_noalloc: fixed buffer not resolved";
        return NMPC_ERR_HIP;
    }
    const hipStream_t caller = static_cast<hipStream_t>(caller_stream);
    unsigned char* base = D.scratch;
    auto at = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
    // the host copy of the descriptor has no control block (each batch places
    // its own); the kernels read the phase from it, so take the problem's
    InstPtrs J = D.hI;
    J.ctl = B.ctl;
    if (!J.ctl || B.ninst != 1) {
        err = "jacobian_u1_x0_noalloc: the problem's own schedule is not set up";
        return NMPC_ERR_HIP;
    }
    J.xp = at(Lo.xp);
    J.bsum = at(Lo.bsum);
    J.uvec = at(Lo.uvec);
    J.adj_rhs = at(Lo.rhs);
    J.adj_w = at(Lo.w);
    J.adj_b = at(Lo.b);
    J.adj_d = at(Lo.d);
    J.adj_lam = at(Lo.lam);
    J.adj_qr = at(Lo.qr);
    J.adj_out = at(Lo.out);
    J.adj_seed = at(Lo.seed);
    InstPtrs* dJ = reinterpret_cast<InstPtrs*>(base + Lo.desc);
    HIP_TRY(join_in(D, caller));
    InstPtrs* const own = B.dI;
    for (int k = 0; k < st.nu; ++k) {
        hipLaunchKernelGGL(k_noalloc_seed, dim3(1), dim3(64), 0, B.stream, J, dJ, k);
        B.dI = dJ;   // the problem's launch schedule over the scratch instance
        launch_adj_seed(B.dI, B.spaces.sp[kSpN], B.stream);
        solve_launches(B, kPredAll, 2);
        launch_adj_refine(0, B.dI, B.spaces, D.adj_eta, B.stream);
        for (int r = 0; r < kAdjRefine; ++r) {
            launch_adj_refine(1, B.dI, B.spaces, D.adj_eta, B.stream);
            solve_launches(B, kPredAll, 3);
            launch_adj_refine(2, B.dI, B.spaces, D.adj_eta, B.stream);
        }
        B.dI = own;
        HIP_TRY(hipGetLastError());
        if (J.gm.pc) {
            launch_x0_map(J.adj_lam, 0, J.gm.pc, jac + (size_t)k * st.nx, st.nx, 1, B.stream);
            HIP_TRY(hipGetLastError());
        } else {
            HIP_TRY(hipMemcpyAsync(jac + (size_t)k * st.nx, J.adj_lam, st.nx * sizeof(double),
                                   hipMemcpyDeviceToDevice, B.stream));
        }
    }
    HIP_TRY(join_out(D, caller));
    return D.adj_eta > 0.0 ? NMPC_REG_FAIL : NMPC_OK;
}

}  // namespace nmpc

namespace nmpc {

// ---- autotuner of the front-kernel variants --------------------------------------------
namespace {

std::mutex g_tune_mutex;
std::unordered_map<uint64_t, std::vector<int>> g_tune_cache;   // structure hash -> variant per factor step

uint64_t fnv(uint64_t h, const void* data, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Hash of everything the factor launches depend on: the supernode partition,
// the row lists and the step sequence.
uint64_t structure_hash(const Problem& p) {
    const Symbolic& sy = p.sym;
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, sy.sn_ptr.data(), sy.sn_ptr.size() * sizeof(int32_t));
    h = fnv(h, sy.sn_rows_ptr.data(), sy.sn_rows_ptr.size() * sizeof(int64_t));
    h = fnv(h, sy.sn_rows.data(), sy.sn_rows.size() * sizeof(int32_t));
    for (const auto& stp : p.dev->fac) h = fnv(h, &stp.kind, sizeof(int));
    return h;
}

void apply_variants(Device& D, const std::vector<int>& v) {
    for (size_t j = 0; j < D.fac.size() && j < v.size(); ++j) D.fac[j].variant = v[j];
    Batch& B = *D.self;
    for (auto& L : B.fac)
        if (L.kind == kStepGroupFactor && L.step < (int)v.size()) L.variant = v[L.step];
    for (int k = 0; k < 4; ++k) {   // the kernels' variants are part of the captured graphs
        if (B.exec[k]) (void)hipGraphExecDestroy(B.exec[k]);
        if (B.graph[k]) (void)hipGraphDestroy(B.graph[k]);
        B.exec[k] = nullptr;
        B.graph[k] = nullptr;
    }
    if (B.loop_exec) (void)hipGraphExecDestroy(B.loop_exec);
    if (B.loop_graph) (void)hipGraphDestroy(B.loop_graph);
    B.loop_exec = nullptr;
    B.loop_graph = nullptr;
}

}  // namespace

nmpc_status device_autotune(Problem& p, int reps, int* changed, std::string& err) {
    Device& D = *p.dev;
    Batch& B = *D.self;
    const uint64_t key = structure_hash(p);
    std::vector<int> best(D.fac.size(), 0);
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) best = it->second;
    }
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        cached = g_tune_cache.count(key) != 0;
    }
    if (!cached) {
        // a symmetric diagonally dominant matrix on the problem's pattern: every
        // variant factors it without failure, and the timing does not depend on values
        const Symbolic& sy = p.sym;
        const int64_t nk = (int64_t)sy.k_orow.size();
        std::vector<double> kv(nk, 0.0), rowsum(p.st.n, 0.0);
        for (int64_t t = 0; t < nk; ++t) {
            if (sy.k_diag[t] >= 0) continue;
            const double v = 0.01 * (double)((t * 2654435761ull) % 1000 + 1) / 1000.0;
            kv[t] = v;
            rowsum[sy.k_orow[t]] += v;
            rowsum[sy.k_ocol[t]] += v;
        }
        for (int64_t t = 0; t < nk; ++t)
            if (sy.k_diag[t] >= 0) kv[t] = 1.0 + rowsum[sy.k_diag[t]];
        HIP_TRY(hipMemcpy(D.hI.kv, kv.data(), nk * sizeof(double), hipMemcpyHostToDevice));
        const size_t nl = B.fac.size();
        std::vector<hipEvent_t> ev(nl + 1);
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
        std::vector<std::vector<double>> t_step(kFactorVariants, std::vector<double>(D.fac.size(), 0.0));
        nmpc_status rc = NMPC_OK;
        for (int v = 0; v < kFactorVariants && rc == NMPC_OK; ++v) {
            std::vector<double> tmin(nl, INFINITY);
            for (int r = 0; r < reps + 1 && rc == NMPC_OK; ++r) {   // the first run warms up
                launch_set_fail(B.dI, 1, 0, B.stream);
                for (size_t i = 0; i < nl; ++i) {
                    BLaunch L = B.fac[i];
                    if (L.kind == kStepGroupFactor) L.variant = v;
                    (void)hipEventRecord(ev[i], B.stream);
                    run_launch(B, L, kPredAll, 0.0, 0);
                }
                (void)hipEventRecord(ev[nl], B.stream);
                if (hipStreamSynchronize(B.stream) != hipSuccess || hipGetLastError() != hipSuccess) {
                    err = "autotune: a factor launch failed";
                    rc = NMPC_ERR_HIP;
                    break;
                }
                if (r == 0) continue;
                for (size_t i = 0; i < nl; ++i) {
                    float ms = 0.0f;
                    if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) tmin[i] = std::min(tmin[i], (double)ms);
                    else (void)hipGetLastError();
                }
            }
            for (size_t i = 0; i < nl; ++i)
                if (B.fac[i].kind == kStepGroupFactor && B.fac[i].step < (int)D.fac.size())
                    t_step[v][B.fac[i].step] += tmin[i];
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        if (rc != NMPC_OK) return rc;
        for (size_t j = 0; j < D.fac.size(); ++j) {
            if (D.fac[j].kind != kStepGroupFactor) continue;
            int bv = 0;
            for (int v = 1; v < kFactorVariants; ++v)
                if (t_step[v][j] < t_step[bv][j]) bv = v;
            best[j] = bv;
        }
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache[key] = best;
    }
    apply_variants(D, best);
    D.adj_ready = false;   // the tuning runs overwrote the factor
    int nchg = 0;
    for (size_t j = 0; j < D.fac.size(); ++j) nchg += D.fac[j].kind == kStepGroupFactor && best[j] != 0;
    if (changed) *changed = nchg;
    return NMPC_OK;
}

}  // namespace nmpc
